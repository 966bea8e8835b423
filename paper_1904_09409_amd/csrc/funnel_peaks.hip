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
// Stage 1: one block per tile of 16 x 256 cells stages the tile and a halo of
//          `radius` cells in LDS (coalesced row loads; the halo wraps, or holds
//          a value that precedes nothing when the border is clamped), flags
//          its local maxima (above the threshold, outside the expansion-border
//          cells), one tile column per thread, from row-window maxima kept in
//          registers, and each wave extracts its first K keys: by one
//          register sort of its keys when it holds at most 128 (the usual
//          case), else by K rounds of a wave-wide minimum; a tile contributes
//          one list per wave.  A wave that held K keys publishes its K-th
//          key as the plane's cutoff (a device-wide minimum): no key after
//          it can be among the plane's first K, since that wave alone holds
//          K earlier ones.  Later waves drop such keys first, so most hold
//          fewer than K and write them unsorted, with no selection at all.
//          Blocks deal the planes round-robin, so every plane's tiles are
//          spread over the whole launch and its cutoff exists after its
//          first few tiles.  For radius 1 on planes of 16-byte aligned rows
//          a second kernel (k_peaks_r1) does the same from registers: one
//          wave per 16-row band of 256 columns, no LDS staging, no block
//          barrier; the selection and the lists are the same.
// Stage 2: a tree of reductions: each block gathers the keys of G lists of
//          K (G K <= 2048) that precede the final cutoff, sorts them and
//          keeps the first K, until one list per plane remains
//          (log_G(tiles) launches, every level spread over the whole GPU).
//          Which keys a stage-1 list holds depends on timing; the cutoff
//          only ever drops keys outside the plane's first K, so the final
//          lists do not.
// Stage 3: one block per plane writes the records.  Lists are built from
//          sorted keys only (the volume detector's LDS gather uses atomics,
//          but sorts what it gathered), so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "fft_core.hpp"
#include "funnel_internal.hpp"

namespace funnel {

constexpr int kTileR = 16, kTileC = 256;  // stage-1 tile: rows x columns of a plane
constexpr int kPeakThreads = 256;           // one tile column per thread
constexpr int kMaxRadius = 8;
constexpr int kHaloC = kTileC + 2 * kMaxRadius;
constexpr int kPadL = kMaxRadius;   // LDS column of the tile's first cell: 16-byte aligned for any radius
constexpr int kMergeLen = 2048;     // keys sorted per stage-2 block
constexpr int kMergeThreads = 256;
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

// Bitonic sort of the first n keys of a (n a power of two, <= the array).
template <int THREADS>
__device__ __forceinline__ void bitonic_sort_n(uint64_t* a, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < n / 2; i += THREADS) {
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
// Sorts 128 keys held by one wave, element lane in a and lane + 64 in b,
// ascending: the bitonic network with lane exchanges by shuffles (no LDS, no
// barriers).  All 64 lanes must be active.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void wave_sort128(uint64_t& a, uint64_t& b, int lane) {
#pragma unroll
  for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride == 64) {   // partners in the same lane (size 128: ascending throughout)
        const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        a = lo;
        b = hi;
        continue;
      }
      const bool low = (lane & stride) == 0;
      const uint64_t pa = shfl_xor_u64(a, stride), pb = shfl_xor_u64(b, stride);
      const bool asc_a = (lane & size) == 0, asc_b = ((lane + 64) & size) == 0;
      a = (low == asc_a) ? (a < pa ? a : pa) : (a < pa ? pa : a);
      b = (low == asc_b) ? (b < pb ? b : pb) : (b < pb ? pb : b);
    }
  }
}

// RADIUS is the neighbourhood radius (1..8), a template parameter so that the
// (2 RADIUS + 1)^2 - 1 comparisons of a cell unroll and their LDS reads are
// all in flight at once.
// Minimum over the 64 lanes of a wave, returned to every lane: within each
// row of 16 lanes by DPP lane permutations (quad swaps, then the half-row and
// row mirrors), then across the four rows by reading one lane of each.  All
// lanes of the wave must be active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm 1,0,3,2
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm 2,3,0,1
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));   // row_mirror
  const uint32_t a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const uint32_t c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return min(min(a, b), min(c, d));
}

// 64-bit keys: the high words first; the low word comes from the one lane
// holding the smallest high word, or (ties) from a second reduction over
// the lanes that hold it
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
  const uint32_t xh = (uint32_t)(x >> 32), xl = (uint32_t)x;
  const uint32_t hi = wave_min_u32(xh);
  const uint64_t holders = __ballot(xh == hi);
  uint32_t lo;
  if (__popcll(holders) == 1) lo = __builtin_amdgcn_readlane(xl, __ffsll((unsigned long long)holders) - 1);
  else lo = wave_min_u32(xh == hi ? xl : 0xffffffffu);
  return ((uint64_t)hi << 32) | lo;
}

// Stage 1's end, per wave: its candidate keys (NS slots per lane, kNoKey
// for none) -> its first K keys at dst.  Keys after the cutoff cmax (a value
// the plane's cutoff `cut` took) go first; the cutoff only decreases and
// every value it takes is safe, so a stale value merely prunes less.  Fewer
// than K are written as they are.  Up
// to 128 keys are packed into the wave's 128 LDS slots `wk` (lanes placed by
// their rank among the wave's keys) and sorted in registers by the shuffle
// bitonic network.  Otherwise each lane sorts its slots, then K rounds of a
// wave-wide minimum over the lanes' first slots; the lane holding the winner
// (keys are unique: exactly one) shifts its slots down.  The last two
// publish their K-th key as the plane's cutoff and return it (the others
// return kNoKey).  All 64 lanes take part.
template <int NS>
__device__ __forceinline__ uint64_t wave_first_k(uint64_t (&mine)[NS], uint64_t* wk, int lane, int K, uint64_t cmax,
                                                 uint64_t* cut, uint64_t* __restrict__ dst) {
#pragma unroll
  for (int j = 0; j < NS; ++j) mine[j] = mine[j] > cmax ? kNoKey : mine[j];
  uint64_t bal[NS];
  int total = 0;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    bal[j] = __ballot(mine[j] != kNoKey);
    total += (int)__popcll(bal[j]);
  }
  if (total < K) {   // uniform over the wave; the reduction sorts
    int base = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal[j] >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal[j], 0u));
      if (mine[j] != kNoKey) dst[base + rank] = mine[j];
      base += (int)__popcll(bal[j]);
    }
    for (int i = total + lane; i < K; i += 64) dst[i] = kNoKey;
    return kNoKey;
  }
  if (total <= 128) {   // uniform over the wave; K <= total
    int base = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal[j] >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal[j], 0u));
      if (mine[j] != kNoKey) wk[base + rank] = mine[j];
      base += (int)__popcll(bal[j]);
    }
    // the wave's LDS writes complete before its lanes read each other's
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint64_t a = lane < total ? wk[lane] : kNoKey;
    uint64_t b = lane + 64 < total ? wk[lane + 64] : kNoKey;
    wave_sort128(a, b, lane);
    if (lane < K) dst[lane] = a;
    if (lane + 64 < K) dst[lane + 64] = b;
    const uint64_t src = K <= 64 ? a : b;   // the K-th key sits in lane (K - 1) mod 64
    const int kl = (K - 1) & 63;
    const uint64_t kth = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(src >> 32), kl) << 32) |
                         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)src, kl);
    if (lane == 0) atomicMin(reinterpret_cast<unsigned long long*>(cut), (unsigned long long)kth);
    return kth;
  }
#pragma unroll
  for (int a = 0; a < NS - 1; ++a)
#pragma unroll
    for (int b = 0; b < NS - 1 - a; ++b) {
      const uint64_t x = mine[b], y = mine[b + 1];
      mine[b] = x < y ? x : y;
      mine[b + 1] = x < y ? y : x;
    }
  uint64_t last = kNoKey;
  for (int k = 0; k < K; ++k) {   // total > 128 and total >= K: every round finds a key
    const uint64_t m = wave_min_u64(mine[0]);
    if (lane == 0) dst[k] = m;
    last = m;
    if (mine[0] == m) {
#pragma unroll
      for (int j = 0; j < NS - 1; ++j) mine[j] = mine[j + 1];
      mine[NS - 1] = kNoKey;
    }
  }
  if (lane == 0) atomicMin(reinterpret_cast<unsigned long long*>(cut), (unsigned long long)last);
  return last;
}

// RADIUS is the neighbourhood radius (1..8), a template parameter so that the
// (2 RADIUS + 1)^2 - 1 comparisons of a cell unroll and their LDS reads are
// all in flight at once.  Output: per tile, one list of K keys per wave (the
// wave's first K local maxima, unordered past the count), [plane][tile][wave][K].
template <int RADIUS>
__global__ void __launch_bounds__(kPeakThreads, 8)
    k_peaks_tile(const float* __restrict__ planes, ImgMap map, PlaneGeom g0, PlaneGeom g1, int nspaces, int nplanes,
                 int tiles, int K, float thr_below, int wrap, int keep_border, uint64_t* __restrict__ cut,
                 uint64_t* __restrict__ out) {
  constexpr int radius = RADIUS;
  constexpr int NW = kPeakThreads / 64;
  __shared__ __align__(16) float val[(kTileR + 2 * RADIUS) * kHaloC];   // |P| of tile and halo; -1: no cell (clamped border)
  const int plane = blockIdx.x % nplanes;       // image * nspaces + space; planes dealt round-robin
  const int img = plane / nspaces, sp = plane % nspaces;
  const PlaneGeom g = sp == 0 ? g0 : g1;
  const float* P = planes + map.out(img) + g.offset;
  const int tcn = (g.cols + kTileC - 1) / kTileC;
  const int ntile = tcn * ((g.rows + kTileR - 1) / kTileR);
  const int tile = blockIdx.x / nplanes;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t* dst = out + (((long long)plane * tiles + tile) * NW + wave) * K;
  if (tile >= ntile) {   // the other space's plane has more tiles
    for (int i = lane; i < K; i += 64) dst[i] = kNoKey;
    return;
  }
  const int r0 = (tile / tcn) * kTileR, c0 = (tile % tcn) * kTileC;
  const int hr = kTileR + 2 * radius;

  // stage the tile and its halo (rows r0-R .. r0+15+R, columns c0-R ..
  // c0+255+R); every load of a thread is issued before the first store
  auto src_row = [&](int lr, bool& in) {   // plane row of halo row lr (wrapped), or !in
    int rr = r0 - radius + lr;
    in = true;
    if (rr < 0 || rr >= g.rows) {
      if (wrap) rr = ((rr % g.rows) + g.rows) % g.rows;
      else in = false;
    }
    return rr;
  };
  const bool vec = c0 + kTileC <= g.cols && (g.cols & 3) == 0 && ((uintptr_t)P & 15) == 0;
  if (vec) {
    // interior columns as 16-byte loads, the 2R side columns one by one
    constexpr int NV = ((kTileR + 2 * radius) * (kTileC / 4) + kPeakThreads - 1) / kPeakThreads;
    constexpr int NS = ((kTileR + 2 * radius) * 2 * radius + kPeakThreads - 1) / kPeakThreads;
    float4 lv[NV];
    bool lin[NV];
    float ls[NS];
    bool lsin[NS];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int i = tid + kPeakThreads * j;
      const int lr = i / (kTileC / 4), q = i % (kTileC / 4);
      bool in;
      int rr = src_row(lr, in);
      in = in && lr < hr;
      lin[j] = in;
      rr = in ? rr : r0;   // loads are unconditional (a row of the tile stands in), so all are in flight at once
      lv[j] = *reinterpret_cast<const float4*>(P + (long long)rr * g.cols + c0 + 4 * q);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int i = tid + kPeakThreads * j;
      const int lr = i / (2 * radius), e = i % (2 * radius);
      int cc = e < radius ? c0 - radius + e : c0 + kTileC + (e - radius);
      bool in;
      const int rr = src_row(lr, in);
      in = in && lr < hr;
      if (cc < 0 || cc >= g.cols) {
        if (wrap) cc = ((cc % g.cols) + g.cols) % g.cols;
        else in = false;
      }
      ls[j] = P[(long long)(in ? rr : r0) * g.cols + (in ? cc : c0)];
      lsin[j] = in;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int i = tid + kPeakThreads * j;
      const int lr = i / (kTileC / 4), q = i % (kTileC / 4);
      if (lr >= hr) continue;
      const float4 x = lv[j];   // -1: a row beyond the clamped border
      *reinterpret_cast<float4*>(val + lr * kHaloC + kPadL + 4 * q) =
          lin[j] ? make_float4(fabsf(x.x), fabsf(x.y), fabsf(x.z), fabsf(x.w)) : make_float4(-1.f, -1.f, -1.f, -1.f);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int i = tid + kPeakThreads * j;
      const int lr = i / (2 * radius), e = i % (2 * radius);
      if (lr >= hr) continue;
      val[lr * kHaloC + kPadL + (e < radius ? e - radius : kTileC + e - radius)] = lsin[j] ? fabsf(ls[j]) : -1.0f;
    }
  } else {
    // hr rows of kHaloC columns from c0 - kPadL (a few more than needed), one by one
    constexpr int NLD = ((kTileR + 2 * radius) * kHaloC + kPeakThreads - 1) / kPeakThreads;
    const int nhalo = hr * kHaloC;
    float ld[NLD];
    bool ldin[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int i = tid + kPeakThreads * j;
      const int lr = i / kHaloC, lc = i % kHaloC;
      int cc = c0 - kPadL + lc;
      bool in;
      const int rr = src_row(lr, in);
      in = in && i < nhalo;
      if (cc < 0 || cc >= g.cols) {
        if (wrap) cc = ((cc % g.cols) + g.cols) % g.cols;
        else in = false;
      }
      ld[j] = P[(long long)(in ? rr : r0) * g.cols + (in ? cc : c0)];   // unconditional: all in flight at once
      ldin[j] = in;
    }
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int i = tid + kPeakThreads * j;
      if (i < nhalo) val[i] = ldin[j] ? fabsf(ld[j]) : -1.0f;
    }
  }
  __syncthreads();

  // local maxima under the order (|P| descending, linear index ascending),
  // down this thread's column of the tile.  For the last 2R+1 halo rows the
  // thread keeps the maximum of the row's 2R+1 cells around its column (mi)
  // and the same without the column's own cell (me), so a cell costs 2R+1
  // LDS reads: a cell above the maximum of its neighbourhood without itself
  // is a peak; a cell equal to it (an exact tie, rare) takes the index
  // tie-break afterwards.  Which cells may be peaks at all (inside the
  // plane, outside the expansion-border bands unless kept) is one bit mask
  // per thread, and the threshold joins the neighbourhood maximum
  // (v >= T is v > thr_below, the float just below T), so each verdict is
  // a few compares and selects.
  constexpr int CPT = kTileR;   // cells per thread
  constexpr int NS = CPT / 2;   // two cells of a column that touch are never both maxima:
  uint32_t khi[NS], klo[NS];    // slot j holds the key of row 2j or 2j+1 if it is one, else kNoKey
#pragma unroll
  for (int j = 0; j < NS; ++j) khi[j] = klo[j] = 0xffffffffu;
  const int lc = tid, c = c0 + lc;
  // per tile row (bit lr): holds cells; lies in a border band (the four
  // centred rows y = e - 2 .. e + 1 around each image edge e = -+himg/2)
  const uint32_t rowok = r0 + CPT <= g.rows ? (1u << CPT) - 1 : (1u << (g.rows - r0)) - 1;
  auto band4 = [&](int first) -> uint32_t {   // bits of tile rows first - r0 .. first - r0 + 3
    const int o = first - r0;
    return o <= -4 || o >= CPT ? 0u : (o >= 0 ? (0xFu << o) : (0xFu >> -o)) & ((1u << CPT) - 1);
  };
  const uint32_t rowband = band4(g.rows / 2 - g.himg / 2 - 2) | band4(g.rows / 2 + g.himg / 2 - 2);
  const int cc = c - g.cols / 2;
  const bool colband = (cc >= -1) & (cc <= 1) & (keep_border == 0);
  const uint32_t cellok = c < g.cols ? (rowok & ~(colband ? rowband : 0u)) : 0u;
  uint32_t idx = (uint32_t)(r0 * g.cols + c);   // linear index of the current cell
  float mi[2 * RADIUS + 1], me[2 * RADIUS + 1];
  auto rowmax = [&](int hr, int j) {
    float m = -1.f;   // -1: clamped border
#pragma unroll
    for (int dc = -radius; dc <= radius; ++dc)
      if (dc != 0) m = fmaxf(m, val[hr * kHaloC + kPadL + lc + dc]);
    me[j] = m;
    mi[j] = fmaxf(m, val[hr * kHaloC + kPadL + lc]);
  };
#pragma unroll
  for (int j = 0; j < 2 * RADIUS; ++j) rowmax(j, j);
  uint32_t ties = 0;
#pragma unroll
  for (int lr = 0; lr < CPT; ++lr) {
    rowmax(lr + 2 * RADIUS, 2 * RADIUS);
    float m = me[RADIUS];
#pragma unroll
    for (int j = 0; j <= 2 * RADIUS; ++j)
      if (j != RADIUS) m = fmaxf(m, mi[j]);
#pragma unroll
    for (int j = 0; j < 2 * RADIUS; ++j) {
      mi[j] = mi[j + 1];
      me[j] = me[j + 1];
    }
    const float v = val[(lr + radius) * kHaloC + kPadL + lc];
    const bool ok = (cellok >> lr) & 1u;
    const bool take = ok & (v > fmaxf(m, thr_below));
    khi[lr / 2] = take ? ~__float_as_uint(v) : khi[lr / 2];   // v >= 0: the key of cell_key
    klo[lr / 2] = take ? idx : klo[lr / 2];
    idx += (uint32_t)g.cols;
    ties |= (ok & (v == m)) ? (1u << lr) : 0u;   // decided below, threshold included
  }
  uint64_t mine[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) mine[j] = ((uint64_t)khi[j] << 32) | klo[j];
  if (ties) {   // equal neighbours: the lower linear index precedes
    uint32_t won = 0;
    for (uint32_t t = ties; t; t &= t - 1) {
      const int lr = __builtin_ctz(t), r = r0 + lr;
      const float v = val[(lr + radius) * kHaloC + kPadL + lc];
      const int idx = r * g.cols + c;
      bool peak = v > thr_below;
      for (int dr = -radius; peak && dr <= radius; ++dr)
        for (int dc = -radius; dc <= radius; ++dc) {
          if (dr == 0 && dc == 0) continue;
          if (val[(lr + radius + dr) * kHaloC + kPadL + lc + dc] != v) continue;
          int rr = r + dr, cc = c + dc;
          rr += rr < 0 ? g.rows : (rr >= g.rows ? -g.rows : 0);
          cc += cc < 0 ? g.cols : (cc >= g.cols ? -g.cols : 0);
          if (rr * g.cols + cc < idx) { peak = false; break; }   // (equal: the cell itself, wrapped)
        }
      won |= peak ? (1u << lr) : 0u;
    }
#pragma unroll
    for (int lr = 0; lr < CPT; ++lr)
      if (won & (1u << lr)) mine[lr / 2] = cell_key(val[(lr + radius) * kHaloC + kPadL + lc], (r0 + lr) * g.cols + c);
  }

  // the sort slots reuse the tile's LDS once every wave has read it
  __syncthreads();
  static_assert(sizeof(uint64_t) * NW * 128 <= sizeof(val), "sort slots exceed the tile's LDS");
  wave_first_k(mine, reinterpret_cast<uint64_t*>(val) + wave * 128, lane, K,
               __hip_atomic_load(cut + plane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), cut + plane, dst);
}

// ---- radius 1: stage 1 from registers
//
// For the default neighbourhood (radius 1) a wave classifies a band of 16
// rows x 256 columns without staging it in LDS: each lane loads its 4
// adjacent columns of the band's 18 rows (one halo row above and below) as
// 16-byte loads, all in flight at once, and one cell of the left (lanes
// 0-17) or right (lanes 32-49) halo column; the neighbours across lanes come
// from DPP wave shifts, into which the halo columns enter at lanes 0 and 63.
// The four waves of a block take four bands stacked down the plane (a 64 x
// 256 tile) and never wait for each other.  Two cells of a 2 x 2 block are
// neighbours, so at most one of them is a maximum: each lane keeps one key
// slot per 2 x 2 block of its 16 x 4 cells, 16 slots at static register
// indices.  The cutoff read at the start joins the threshold, so a key
// after it is never taken; cells equal to their neighbourhood maximum or to
// that bound (rare) are decided from global memory afterwards, by the
// order's index tie-break and the exact cutoff key.  Wrapping reaches every
// neighbour in one step for planes of at least 32 rows and 128 columns, and
// the 16-byte loads need planes whose rows, plane offsets and base are
// multiples of 4 floats; the launch takes this kernel only for those.
constexpr int kR1Band = 16;                                // rows per wave
constexpr int kR1TileR = kR1Band * (kPeakThreads / 64);    // rows per block
constexpr int kR1TileC = 256;                              // 4 columns per lane

int peaks_r1_tiles(int rows, int cols) {
  return ((rows + kR1TileR - 1) / kR1TileR) * ((cols + kR1TileC - 1) / kR1TileC);
}

// The bits of |q| as an int (>= 0, ordered as the floats), or -1 for an
// absent cell or a NaN (bits above infinity's): such a cell never blocks a
// neighbour and is never a peak, as under float comparisons.  The presence
// test selects a limit rather than the loaded value: a select between a
// load and a constant becomes a branch around the load and a wait for it.
__device__ __forceinline__ int cell_bits(float q, bool present) {
  const uint32_t b = __float_as_uint(q) & 0x7fffffffu;
  const int lim = present ? 0x7f800000 : -1;
  return (int)b <= lim ? (int)b : -1;
}

// lane i receives x of lane i - 1 (wave_shr:1); lane 0 receives `edge`
__device__ __forceinline__ int from_prev_lane(int edge, int x) {
  return __builtin_amdgcn_update_dpp(edge, x, 0x138, 0xF, 0xF, false);
}
// lane i receives x of lane i + 1 (wave_shl:1); lane 63 receives `edge`
__device__ __forceinline__ int from_next_lane(int edge, int x) {
  return __builtin_amdgcn_update_dpp(edge, x, 0x130, 0xF, 0xF, false);
}

// A plane coordinate one step outside [0, n) wrapped back (wrap) or marked
// absent (!in); one step suffices for |excess| < n.
__device__ __forceinline__ int wrap1(int c, int n, int wrap, bool& in) {
  const bool lo = c < 0, hi = c >= n;
  in = in && (wrap || !(lo || hi));
  return lo ? c + n : (hi ? c - n : c);
}

// The exact radius-1 verdict on cell (r, c) of plane P (inside it): at or
// above the threshold, not after the cutoff key, and preceding each of its 8
// neighbours (present ones: wrapped, or none beyond a clamped border) in the
// order |P| descending, linear index ascending.
__device__ bool r1_exact_peak(const float* __restrict__ P, int rows, int cols, int r, int c, int wrap,
                              float thr_below, uint64_t cmax) {
  const uint32_t idx = (uint32_t)(r * cols + c);
  const float v = fabsf(P[idx]);
  if (!(v > thr_below) || cell_key(v, (int)idx) > cmax) return false;
  for (int dr = -1; dr <= 1; ++dr)
    for (int dc = -1; dc <= 1; ++dc) {
      if (dr == 0 && dc == 0) continue;
      bool in = true;
      const int rr = wrap1(r + dr, rows, wrap, in), cc = wrap1(c + dc, cols, wrap, in);
      if (!in) continue;
      const uint32_t j = (uint32_t)(rr * cols + cc);
      const float u = fabsf(P[j]);
      if (u > v || (u == v && j < idx)) return false;
    }
  return true;
}

__global__ void __launch_bounds__(kPeakThreads, 4)
    k_peaks_r1(const float* __restrict__ planes, ImgMap map, PlaneGeom g0, PlaneGeom g1, int nspaces, int nplanes,
               int tiles, int K, float thr_below, int wrap, int keep_border, uint64_t* __restrict__ cut,
               uint64_t* __restrict__ out) {
  constexpr int NW = kPeakThreads / 64, HR = kR1Band + 2, NS = kR1Band / 2 * 2;
  __shared__ uint64_t wkeys[NW][128];   // the register sort's staging
  const int plane = blockIdx.x % nplanes;   // planes dealt round-robin
  const int img = plane / nspaces, sp = plane % nspaces;
  const PlaneGeom g = sp == 0 ? g0 : g1;
  const int rows = g.rows, cols = g.cols;
  const float* P = planes + map.out(img) + g.offset;
  const int tcn = (cols + kR1TileC - 1) / kR1TileC;
  const int ntile = tcn * ((rows + kR1TileR - 1) / kR1TileR);
  const int tile = blockIdx.x / nplanes;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t* dst = out + (((long long)plane * tiles + tile) * NW + wave) * K;
  // Row tiles from the plane's centre outwards.  Any order gives the same
  // lists; this one publishes high cutoffs first, because a parameter
  // plane's strongest cells lie in its central rows (where the image itself
  // maps), so later bands keep fewer keys.
  const int nrt = (rows + kR1TileR - 1) / kR1TileR, t = tile / tcn;
  const int rt = nrt / 2 + ((t & 1) ? -((t + 1) >> 1) : (t >> 1));   // a permutation of 0 .. nrt-1
  const int r0 = rt * kR1TileR + wave * kR1Band, c0 = (tile % tcn) * kR1TileC;
  if (tile >= ntile || r0 >= rows) {   // the other space's plane has more tiles, or a band past the last row
    for (int i = lane; i < K; i += 64) dst[i] = kNoKey;
    return;
  }

  // the plane's cutoff, read before the cells (loads complete in order)
  const uint64_t cmax = __hip_atomic_load(cut + plane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // Cells are compared as the bits of |P| (an int order equal to the float
  // order for |P| >= 0), -1 for an absent cell or a NaN.  Band rows lr = 0
  // .. 17 are plane rows r0 - 1 + lr, wrapped or absent; the lane's columns
  // cb .. cb + 3 wrap past the right edge to cb - cols < cols (cols >= 128)
  // and lie on one side of it (cols is a multiple of 4).  Absent cells read
  // row r0, column 0.
  const int cb = c0 + 4 * lane;
  auto row_ptr = [&](int lr, bool& rin) {   // uniform: SGPRs
    rin = true;
    const int rr = wrap1(r0 - 1 + lr, rows, wrap, rin);
    return P + (long long)(rin ? rr : r0) * cols;
  };
  // halo columns c0 - 1 (lanes 0-17, row lane) and c0 + 256 (lanes 32-49,
  // row lane - 32); c0 + 256 - cols may reach cols once.  Issued first: the
  // first row needs it.
  int hal;
  {
    const int lr = lane & 31;
    bool in = lr < HR;
    int c = lane < 32 ? c0 - 1 : c0 + kR1TileC;
    c = wrap1(c, cols, wrap, in);
    c = c >= cols ? c - cols : c;
    const int rr = wrap1(r0 - 1 + lr, rows, wrap, in);
    hal = cell_bits(P[(long long)(in ? rr : r0) * cols + (in ? c : 0)], in);
  }
  float4 raw[HR];
  bool rowin[HR];
  bool cin = true;
  {
    const int cw = wrap1(cb, cols, wrap, cin);
    const uint32_t co = cin ? (uint32_t)cw : 0u;   // one 32-bit column offset per lane, for every row
#pragma unroll
    for (int lr = 0; lr < HR; ++lr) {
      // unconditional loads (an absent cell reads column 0) keep all in flight
      const float* rp = row_ptr(lr, rowin[lr]);
      raw[lr] = *reinterpret_cast<const float4*>(rp + co);
    }
  }
  // row lr as cell bits, converted where it is first used (rows arrive in order)
  int x[HR][4];
  auto convert = [&](int lr) {
    const bool in = rowin[lr] && cin;
    x[lr][0] = cell_bits(raw[lr].x, in);
    x[lr][1] = cell_bits(raw[lr].y, in);
    x[lr][2] = cell_bits(raw[lr].z, in);
    x[lr][3] = cell_bits(raw[lr].w, in);
  };

  // a key precedes the cutoff key cmax when |P| exceeds the value part of
  // cmax: that value joins the threshold (bits; -1 when negative: every
  // |P| >= 0 passes); cells equal to it go to the exact check below
  const float thr_w = cmax == kNoKey ? thr_below : fmaxf(thr_below, __uint_as_float(~(uint32_t)(cmax >> 32)));
  const int thr_i = thr_w < 0.f ? -1 : (int)__float_as_uint(thr_w);

  // which cells may be peaks: rows inside the plane (bit cr of the band),
  // columns inside it, and not both in a border row band (four centred rows
  // y = e - 2 .. e + 1 around each image edge e = -+himg/2) and within one
  // column of the centre column, unless the border is kept.  A cell that may
  // not be a peak gets the bound INT_MAX, above every |P|.
  const uint32_t rowok = r0 + kR1Band <= rows ? (1u << kR1Band) - 1 : (1u << (rows - r0)) - 1;
  auto band4 = [&](int first) -> uint32_t {   // bits of band rows first - r0 .. first - r0 + 3
    const int o = first - r0;
    return o <= -4 || o >= kR1Band ? 0u : (o >= 0 ? (0xFu << o) : (0xFu >> -o)) & ((1u << kR1Band) - 1);
  };
  const uint32_t bandrows = keep_border ? 0u : (band4(rows / 2 - g.himg / 2 - 2) | band4(rows / 2 + g.himg / 2 - 2));
  bool colok[4], colband[4];
  int thc[4], thb[4];   // bound of column j in a plain row, in a border-band row
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    colok[j] = cb + j < cols;
    const int cc = cb + j - cols / 2;
    colband[j] = cc >= -1 && cc <= 1;
    thc[j] = colok[j] ? thr_i : INT_MAX;
    thb[j] = colok[j] && !colband[j] ? thr_i : INT_MAX;
  }

  // row maxima: me = the larger horizontal neighbour, mi = with the cell
  auto rowmax = [&](int lr, int (&me)[4], int (&mi)[4]) {
    convert(lr);
    const int left = from_prev_lane(__builtin_amdgcn_readlane(hal, lr), x[lr][3]);
    const int right = from_next_lane(__builtin_amdgcn_readlane(hal, 32 + lr), x[lr][0]);
    me[0] = max(left, x[lr][1]);
    me[1] = max(x[lr][0], x[lr][2]);
    me[2] = max(x[lr][1], x[lr][3]);
    me[3] = max(x[lr][2], right);
#pragma unroll
    for (int j = 0; j < 4; ++j) mi[j] = max(me[j], x[lr][j]);
  };
  int sv[NS];         // slot (cr / 2) * 2 + j / 2: |P| bits of its maximum, -1 for none
  uint32_t so = 0;    // bits 2k, 2k + 1: the maximum's place in slot k's 2 x 2 block, 2 dr + dc
#pragma unroll
  for (int k = 0; k < NS; ++k) sv[k] = -1;
  int miP[4], meC[4], miC[4], tmp[4];
  rowmax(0, tmp, miP);
  rowmax(1, meC, miC);
  uint32_t tierows = 0;
#pragma unroll
  for (int cr = 0; cr < kR1Band; ++cr) {   // cell row cr: plane row r0 + cr, band row cr + 1
    int meN[4], miN[4];
    rowmax(cr + 2, meN, miN);
    const bool rok = (rowok >> cr) & 1u, rband = (bandrows >> cr) & 1u;
    bool tie = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int v = x[cr + 1][j];
      const int th = rok ? (rband ? thb[j] : thc[j]) : INT_MAX;
      const int m = max(max(miP[j], meC[j]), max(miN[j], th));
      const bool take = v > m;
      tie |= v == m;
      const int k = (cr / 2) * 2 + j / 2;
      sv[k] = take ? v : sv[k];
      so = take ? (so & ~(3u << 2 * k)) | ((uint32_t)((cr & 1) * 2 + (j & 1)) << 2 * k) : so;
    }
    tierows |= tie ? (1u << cr) : 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      miP[j] = miC[j];
      meC[j] = meN[j];
      miC[j] = miN[j];
    }
    // row by row, in load order: keeps the scheduler from starting on the
    // last rows (and waiting for every load) first
    __builtin_amdgcn_sched_barrier(0);
  }
  if (__ballot(tierows != 0)) {   // exact verdicts on the rows with a tie (any lane)
    uint64_t won = 0;
    for (uint32_t t = tierows; t; t &= t - 1) {
      const int cr = __builtin_ctz(t);
      const bool rband = (bandrows >> cr) & 1u;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (colok[j] && !(rband && colband[j]) && r1_exact_peak(P, rows, cols, r0 + cr, cb + j, wrap, thr_below, cmax))
          won |= 1ull << (cr * 4 + j);
    }
    if (won) {
#pragma unroll
      for (int cr = 0; cr < kR1Band; ++cr)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if ((won >> (cr * 4 + j)) & 1u) {
            const int k = (cr / 2) * 2 + j / 2;
            sv[k] = (int)(__float_as_uint(P[(long long)(r0 + cr) * cols + cb + j]) & 0x7fffffffu);
            so = (so & ~(3u << 2 * k)) | ((uint32_t)((cr & 1) * 2 + (j & 1)) << 2 * k);
          }
    }
  }
  uint64_t mine[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const uint32_t first = (uint32_t)((r0 + 2 * (k / 2)) * cols + cb + 2 * (k % 2));
    const uint32_t place = (so >> 2 * k) & 3u;
    const uint32_t idx = first + (place >> 1) * (uint32_t)cols + (place & 1u);
    mine[k] = sv[k] < 0 ? kNoKey : ((uint64_t)(~(uint32_t)sv[k]) << 32) | idx;
  }
  // a fresh read of the cutoff prunes more of the keys
  wave_first_k(mine, wkeys[wave], lane, K, __hip_atomic_load(cut + plane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
               cut + plane, dst);
}

__global__ void k_fill_keys(uint64_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = kNoKey;
}

// Lists [plane][nin][K] -> [plane][nout][K], nout = ceil(nin / G): block
// (j, plane) gathers the keys of lists j G .. j G + G - 1 that are present
// and not after the plane's cutoff (cut: NULL for none), sorts them and
// keeps the first K.  Before the last level (nout > 1) at most K gathered
// keys pass on unsorted: only the last level's list has to be in order.
__global__ void __launch_bounds__(kMergeThreads)
    k_peaks_reduce(const uint64_t* __restrict__ in, int nin, uint64_t* __restrict__ out, int nout, int K, int G,
                   const uint64_t* __restrict__ cut) {
  __shared__ uint64_t keys[kMergeLen];
  __shared__ int count;
  const int plane = blockIdx.y, j = blockIdx.x, lane = threadIdx.x & 63;
  const uint64_t* src = in + ((long long)plane * nin + (long long)j * G) * K;
  const int avail = (nin - j * G < G ? nin - j * G : G) * K;
  const uint64_t cmax = cut ? cut[plane] : kNoKey;   // stage 1 has ended: final
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  for (int i0 = 0; i0 < avail; i0 += kMergeThreads) {   // same trip count for every lane
    const int i = i0 + threadIdx.x;
    const uint64_t key = i < avail ? src[i] : kNoKey;
    const bool keep = key != kNoKey && key <= cmax;
    const uint64_t bal = __ballot(keep);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(&count, (int)__popcll(bal));
    base = __shfl(base, 0, 64);
    if (keep) keys[base + rank] = key;
  }
  __syncthreads();
  const int c = count;
  uint64_t* dst = out + ((long long)plane * nout + j) * K;
  if (nout > 1 && c <= K) {   // uniform: all of them go on, unsorted (the last level sorts)
    for (int i = threadIdx.x; i < K; i += kMergeThreads) dst[i] = i < c ? keys[i] : kNoKey;
    return;
  }
  int n = 1;   // sort the keys gathered, padded to a power of two (>= K, <= G K)
  while (n < c || n < K) n <<= 1;
  for (int i = c + threadIdx.x; i < n; i += kMergeThreads) keys[i] = kNoKey;
  __syncthreads();
  bitonic_sort_n<kMergeThreads>(keys, n);
  for (int i = threadIdx.x; i < K; i += kMergeThreads) dst[i] = keys[i];
}

// One sorted list of K keys per plane -> records and counts.
__global__ void __launch_bounds__(kMergeThreads)
    k_peaks_records(const float* __restrict__ planes, ImgMap map, const int* __restrict__ gidx, PlaneGeom g0,
                    PlaneGeom g1, int nspaces, int space0, int K, const uint64_t* __restrict__ list,
                    ft_peak* __restrict__ peaks, int32_t* __restrict__ n_found) {
  const int plane = blockIdx.x;
  const int img = plane / nspaces, sp = plane % nspaces;
  const int gimg = gidx ? gidx[img] : img;
  const PlaneGeom g = sp == 0 ? g0 : g1;
  const float* P = planes + map.out(img) + g.offset;
  const uint64_t* keys = list + (long long)plane * K;
  ft_peak* dst = peaks + ((long long)gimg * nspaces + sp) * K;
  for (int i = threadIdx.x; i < K; i += kMergeThreads) {
    if (keys[i] == kNoKey) continue;
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
  if (threadIdx.x == 0) {
    int count = 0;   // sorted: the valid keys come first
    while (count < K && keys[count] != kNoKey) ++count;
    n_found[(long long)gimg * nspaces + sp] = count;
  }
}

// lists merged per stage-2 block
static int merge_group(int K) { return kMergeLen / K > 1 ? kMergeLen / K : 2; }

// stage-1 lists, then the first reduction level's lists (later levels reuse
// the first buffer, which is large enough for them), then one cutoff key per
// plane
size_t peaks_workspace_bytes(int nplanes_total, int tiles, int K) {
  const size_t lists = (size_t)tiles * (kPeakThreads / 64);
  const size_t lvl1 = (lists + merge_group(K) - 1) / merge_group(K);
  return (size_t)nplanes_total * ((lists + lvl1) * (size_t)K + 1) * sizeof(uint64_t);
}

// Reduce `lists` key lists per plane to one, ping-ponging between the stage-1
// buffer `cand` and the level-1 buffer behind it; *out: the final lists.
static hipError_t reduce_lists(uint64_t* cand, int planes_n, int lists, int K, const uint64_t* cut,
                               const uint64_t** out, hipStream_t s) {
  const int G = merge_group(K);
  uint64_t* bufs[2] = {cand, cand + (size_t)planes_n * lists * K};
  int cur = 0, n = lists;
  do {
    const int nout = (n + G - 1) / G;
    k_peaks_reduce<<<dim3(nout, planes_n), kMergeThreads, 0, s>>>(bufs[cur], n, bufs[1 - cur], nout, K, G, cut);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur = 1 - cur;
    n = nout;
  } while (n > 1);
  *out = bufs[cur];
  return hipSuccess;
}

static int peaks_tiles_lds(int rows, int cols) {
  return ((rows + kTileR - 1) / kTileR) * ((cols + kTileC - 1) / kTileC);
}
// in units of kPeakThreads / 64 lists per plane: the larger need of the two stage-1 kernels
int peaks_tiles(int rows, int cols) {
  const int a = peaks_tiles_lds(rows, cols), b = peaks_r1_tiles(rows, cols);
  return a > b ? a : b;
}

hipError_t launch_peaks(const float* planes, ImgMap map, const int* gidx, int batch, int nspaces, int space0,
                        const int* rows, const int* cols, const int* himg, const long long* offset, int K, float thr,
                        int radius, int wrap, int keep_border, ft_peak* peaks, int32_t* n_found, void* ws,
                        hipStream_t s) {
  PlaneGeom g[2];
  // radius 1 on planes of at least 32 x 128 cells, 16-byte aligned rows:
  // the register kernel (per-image offsets from a table are multiples of 4
  // floats: ragged plans check their descriptors for it)
  bool r1 = radius == 1 && ((uintptr_t)planes & 15) == 0 && (map.out_off || (map.out_stride & 3) == 0);
  for (int i = 0; i < nspaces; ++i)
    r1 = r1 && rows[i] >= 32 && cols[i] >= 128 && (cols[i] & 3) == 0 && (offset[i] & 3) == 0;
  int tiles = 0;
  for (int i = 0; i < nspaces; ++i) {
    g[i] = PlaneGeom{rows[i], cols[i], himg[i], offset[i]};
    const int t = r1 ? peaks_r1_tiles(rows[i], cols[i]) : peaks_tiles_lds(rows[i], cols[i]);
    tiles = t > tiles ? t : tiles;
  }
  if (nspaces == 1) g[1] = g[0];
  if (radius < 1 || radius > kMaxRadius) return hipErrorInvalidValue;
  const int planes_n = batch * nspaces;
  // lists per plane: one per wave of a tile (peaks_tiles sizes the
  // workspace for the larger count of the two kernels)
  const size_t lists = (size_t)tiles * (kPeakThreads / 64);
  const size_t lvl1 = (lists + merge_group(K) - 1) / merge_group(K);
  uint64_t* cand = static_cast<uint64_t*>(ws);
  uint64_t* cut = cand + (size_t)planes_n * (lists + lvl1) * K;   // as peaks_workspace_bytes lays it out
  k_fill_keys<<<(planes_n + 255) / 256, 256, 0, s>>>(cut, planes_n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid1((unsigned)(tiles * planes_n));
  const float thr_below = std::nextafter(thr, -INFINITY);   // v >= thr  <=>  v > thr_below
  if (r1) {
    k_peaks_r1<<<grid1, kPeakThreads, 0, s>>>(planes, map, g[0], g[1], nspaces, planes_n, tiles, K, thr_below, wrap,
                                              keep_border, cut, cand);
  } else {
    switch (radius) {
#define CASE(R)                                                                                              \
  case R:                                                                                                    \
    k_peaks_tile<R><<<grid1, kPeakThreads, 0, s>>>(planes, map, g[0], g[1], nspaces, planes_n, tiles, K, thr_below, \
                                                   wrap, keep_border, cut, cand);                            \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t* list = nullptr;
  e = reduce_lists(cand, planes_n, (int)lists, K, cut, &list, s);   // one list per wave of every tile
  if (e != hipSuccess) return e;
  k_peaks_records<<<planes_n, kMergeThreads, 0, s>>>(planes, map, gidx, g[0], g[1], nspaces, space0, K, list, peaks,
                                                     n_found);
  return hipGetLastError();
}


// ------------------------------------------------------------------ volumes (App. A)
//
// The same detector on the parameter volume of the volume transform: a cell
// is detected when it precedes every other cell of its (2R+1)^3
// neighbourhood (toroidal, or clamped), is >= the threshold and is not one
// of the cells where the expansion's front and back faces focus.  Stage-1
// tiles are 8 slices x 4 rows x 64 columns: each thread walks one column of
// the tile through the 8 slices over the LDS copy of the tile and its halo,
// keeping the window maxima of the last 2R+1 slices in registers, so a cell
// costs (2R+1)^2 LDS reads; the block's local maxima are then gathered in
// LDS and sorted once, and the block emits its first K.  Eight slices keep
// the LDS copy at 16 KB (R = 1), so eight blocks share a compute unit and
// hide each other's load latency (16 slices: five blocks, 25 % slower).
// Stages 2 and 3 as for planes.
constexpr int kVTileZ = 8, kVTileY = kPeakThreads / 64, kVTileX = 64;
constexpr int kMaxVRadius = 2;

struct VolGeom {
  int nz, ny, nx;      // parameter volume: Nzp x Ny x Nx
  int zimg;            // depth Nz of the transformed volume (its faces focus at z = -+Nz/2)
  long long stride;    // floats per parameter volume
};

// Coordinate c of a halo cell on an axis of n cells: wrapped once (R < n and
// the tile starts inside the volume, so one step reaches every cell a real
// cell needs; cells beyond those are clamped and never used), or !in when
// the border is clamped.  Selects only, no branches.
__device__ __forceinline__ int halo_coord(int c, int n, int wrap, bool& in) {
  const bool lo = c < 0, hi = c >= n;
  in = in & ((wrap != 0) | !(lo | hi));
  const int w = lo ? c + n : (hi ? c - n : c);
  return w < n - 1 ? (w > 0 ? w : 0) : n - 1;
}

// Tile geometry and the staging of one tile plus its halo: HZ * HY rows of
// HX cells, |P| in LDS (-1: no cell, beyond a clamped border).  A row's cell
// x0 sits at column PX, so rows and their 16-byte stores are aligned.
template <int R>
struct VTile {
  static constexpr int PX = 4;
  static_assert(R <= PX, "halo wider than the row padding");
  static constexpr int HZ = kVTileZ + 2 * R, HY = kVTileY + 2 * R, HX = kVTileX + 2 * PX;
  static constexpr int NH = HZ * HY * HX;
  static constexpr int NV = (HZ * HY * (kVTileX / 4) + kPeakThreads - 1) / kPeakThreads;   // 16-byte loads
  static constexpr int NSD = (HZ * HY * 2 * R + kPeakThreads - 1) / kPeakThreads;         // side cells
  static constexpr int NLD = (NH + kPeakThreads - 1) / kPeakThreads;                     // scalar path
  static constexpr int NSLOT = kVTileZ / 2;
  static_assert(NH * sizeof(float) >= kPeakThreads * NSLOT * sizeof(uint64_t), "key space");

  struct Origin {
    int vol, tile, x0, y0, z0;
  };
  __device__ static Origin origin(const VolGeom& g, int tiles, int t) {
    const int tx = (g.nx + kVTileX - 1) / kVTileX, ty = (g.ny + kVTileY - 1) / kVTileY;
    const int tile = t % tiles;
    return Origin{t / tiles, tile, (tile % tx) * kVTileX, ((tile / tx) % ty) * kVTileY, (tile / (tx * ty)) * kVTileZ};
  }
  // offset of the tile's first row (z0, y0), cell x = 0
  __device__ static long long origin_row(const VolGeom& g, const Origin& o) {
    return ((long long)o.z0 * g.ny + o.y0) * g.nx;
  }
  // offset of halo row r's cell x = 0 (in: the row exists)
  __device__ static long long row_base(const VolGeom& g, const Origin& o, int wrap, int r, bool& in) {
    in = r < HZ * HY;
    const int z = halo_coord(o.z0 - R + r / HY, g.nz, wrap, in);
    const int y = halo_coord(o.y0 - R + r % HY, g.ny, wrap, in);
    return ((long long)z * g.ny + y) * g.nx;
  }

  // 16-byte path (the tile's 64 columns inside the volume, rows 16-byte aligned)
  struct Regs {
    float4 lv[NV];
    bool lin[NV];
    float ls[NSD];
    bool lsin[NSD];
  };
  __device__ static void load_vec(const float* P, const VolGeom& g, const Origin& o, int wrap, Regs& q) {
    const int tid = threadIdx.x;
    // most tiles' halo rows lie inside the volume along z and y (uniform over
    // the block): their offsets need no wrapping or clamping
    const bool interior = o.z0 >= R && o.z0 + kVTileZ + R <= g.nz && o.y0 >= R && o.y0 + kVTileY + R <= g.ny;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int i = tid + kPeakThreads * j, r = i / (kVTileX / 4), c = i % (kVTileX / 4);
      bool in;
      long long b;
      if (interior) {
        in = (HZ * HY * (kVTileX / 4)) % kPeakThreads == 0 || r < HZ * HY;
        b = ((long long)(o.z0 - R + r / HY) * g.ny + (o.y0 - R + r % HY)) * g.nx;
      } else {
        b = row_base(g, o, wrap, r, in);
      }
      q.lin[j] = in;
      // unconditional, so all are in flight at once; a lane with nothing to
      // stage reads the tile's own first row, which the block fetches anyway
      q.lv[j] = *reinterpret_cast<const float4*>(P + (in ? b : origin_row(g, o)) + o.x0 + 4 * c);
    }
#pragma unroll
    for (int j = 0; j < NSD; ++j) {
      const int i = tid + kPeakThreads * j, r = i / (2 * R), e = i % (2 * R);
      bool in;
      long long b;
      if (interior) {
        in = r < HZ * HY;
        b = ((long long)(o.z0 - R + r / HY) * g.ny + (o.y0 - R + r % HY)) * g.nx;
      } else {
        b = row_base(g, o, wrap, r, in);
      }
      const int x = halo_coord(e < R ? o.x0 - R + e : o.x0 + kVTileX + (e - R), g.nx, wrap, in);
      q.ls[j] = P[in ? b + x : origin_row(g, o) + o.x0];
      q.lsin[j] = in;
    }
  }
  __device__ static void store_vec(float* val, const Regs& q) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int i = tid + kPeakThreads * j, r = i / (kVTileX / 4), c = i % (kVTileX / 4);
      if ((HZ * HY * (kVTileX / 4)) % kPeakThreads != 0 && r >= HZ * HY) continue;
      const float4 x = q.lv[j];
      *reinterpret_cast<float4*>(val + r * HX + PX + 4 * c) =
          q.lin[j] ? make_float4(fabsf(x.x), fabsf(x.y), fabsf(x.z), fabsf(x.w)) : make_float4(-1.f, -1.f, -1.f, -1.f);
    }
#pragma unroll
    for (int j = 0; j < NSD; ++j) {
      const int i = tid + kPeakThreads * j, r = i / (2 * R), e = i % (2 * R);
      if ((HZ * HY * 2 * R) % kPeakThreads != 0 && r >= HZ * HY) continue;
      val[r * HX + PX + (e < R ? e - R : kVTileX + e - R)] = q.lsin[j] ? fabsf(q.ls[j]) : -1.0f;
    }
  }
  // any tile: cell by cell, every load issued before the first store
  __device__ static void stage_scalar(float* val, const float* P, const VolGeom& g, const Origin& o, int wrap) {
    const int tid = threadIdx.x;
    float ld[NLD];
    bool ldin[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int i = tid + kPeakThreads * j;
      bool in;
      const long long b = row_base(g, o, wrap, i / HX, in);
      const int xc = o.x0 - PX + i % HX;   // the padding columns beyond the halo are staged too
      in = in & (xc >= o.x0 - R) & (xc < o.x0 + kVTileX + R);
      const int x = halo_coord(xc, g.nx, wrap, in);
      ld[j] = P[in ? b + x : origin_row(g, o) + o.x0];   // unconditional: all in flight at once
      ldin[j] = in;
    }
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int i = tid + kPeakThreads * j;
      if (NH % kPeakThreads == 0 || i < NH) val[i] = ldin[j] ? fabsf(ld[j]) : -1.0f;
    }
  }
};

// The local maxima of a staged tile and the tile's first K keys, written to
// dst.  Every thread of the block calls it; it leaves val overwritten (the
// block's keys) and returns without a final barrier.
template <int R>
__device__ void vtile_detect(float* val, int* nkeys, const VolGeom& g, const typename VTile<R>::Origin& o, int K,
                             float thr_below, int keep_border, uint64_t* cut, uint64_t* dst) {
  using T = VTile<R>;
  constexpr int HY = T::HY, HX = T::HX, NS = T::NSLOT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x0 = o.x0, y0 = o.y0, z0 = o.z0;

  // Walk down the thread's column of the tile with, for the last 2R+1 halo
  // slices, the maximum of the (2R+1)^2 window around the column (m9) and the
  // same without the column's own cell (m8).  A cell above the maximum of
  // its neighbourhood without itself is a peak; a cell equal to it (an exact
  // tie, rare) is resolved afterwards by the index tie-break.  The verdicts
  // are selects, so the loop has no divergent branches.
  uint64_t mine[NS];   // two cells adjacent along z are never both maxima: slot lz / 2
  uint32_t khi[NS], klo[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) khi[j] = klo[j] = 0xffffffffu;
  const int x = x0 + lane, y = y0 + wave;
  // which of the column's cells may be peaks (bit lz): inside the volume and,
  // unless kept, outside the expansion faces (four centred slices around
  // each image face, at slope bins -1..1 in both x and y); the threshold
  // joins the neighbourhood maximum (v >= T is v > thr_below)
  constexpr uint32_t kAll = (1u << kVTileZ) - 1;
  const uint32_t zok = z0 + kVTileZ <= g.nz ? kAll : (1u << (g.nz - z0)) - 1;
  auto band4 = [&](int first) -> uint32_t {   // bits of tile slices first - z0 .. first - z0 + 3
    const int o4 = first - z0;
    return o4 <= -4 || o4 >= kVTileZ ? 0u : (o4 >= 0 ? (0xFu << o4) : (0xFu >> -o4)) & kAll;
  };
  const uint32_t zband = band4(g.nz / 2 - g.zimg / 2 - 2) | band4(g.nz / 2 + g.zimg / 2 - 2);
  const int cx = x - g.nx / 2, cy = y - g.ny / 2;
  const bool center = (cx >= -1) & (cx <= 1) & (cy >= -1) & (cy <= 1) & (keep_border == 0);
  const uint32_t cellok = (x < g.nx) & (y < g.ny) ? (zok & ~(center ? zband : 0u)) : 0u;
  uint32_t idx = (uint32_t)((z0 * g.ny + y) * g.nx + x);   // linear index of the current cell
  const int lc = (wave + R) * HX + lane + T::PX;   // this column's cell in a halo slice
  float m9[2 * R + 1], m8[2 * R + 1];
  auto window = [&](int hz, int j) {
    float m = -1.f;
#pragma unroll
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll
      for (int dx = -R; dx <= R; ++dx)
        if (dy != 0 || dx != 0) m = fmaxf(m, val[hz * HY * HX + lc + dy * HX + dx]);
    m8[j] = m;
    m9[j] = fmaxf(m, val[hz * HY * HX + lc]);
  };
#pragma unroll
  for (int j = 0; j < 2 * R; ++j) window(j, j);
  uint32_t ties = 0;
#pragma unroll
  for (int lz = 0; lz < kVTileZ; ++lz) {
    window(lz + 2 * R, 2 * R);
    float m = m8[R];
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j)
      if (j != R) m = fmaxf(m, m9[j]);
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) {
      m9[j] = m9[j + 1];
      m8[j] = m8[j + 1];
    }
    const float v = val[(lz + R) * HY * HX + lc];
    const bool ok = (cellok >> lz) & 1u;
    const bool take = ok & (v > fmaxf(m, thr_below));
    khi[lz / 2] = take ? ~__float_as_uint(v) : khi[lz / 2];   // v >= 0: the key of cell_key
    klo[lz / 2] = take ? idx : klo[lz / 2];
    idx += (uint32_t)(g.ny * g.nx);
    ties |= (ok & (v == m)) ? (1u << lz) : 0u;   // decided below, threshold included
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) mine[j] = ((uint64_t)khi[j] << 32) | klo[j];
  if (ties) {   // equal neighbours: the lower linear index precedes
    uint32_t won = 0;
    for (uint32_t t = ties; t; t &= t - 1) {
      const int lz = __builtin_ctz(t), z = z0 + lz;
      const int c = (lz + R) * HY * HX + lc;
      const float v = val[c];
      const int idx = (z * g.ny + y) * g.nx + x;
      bool peak = v > thr_below;
      for (int dz = -R; peak && dz <= R; ++dz)
        for (int dy = -R; peak && dy <= R; ++dy)
          for (int dx = -R; dx <= R; ++dx) {
            if ((dz == 0 && dy == 0 && dx == 0) || val[c + (dz * HY + dy) * HX + dx] != v) continue;
            int zz = z + dz, yy = y + dy, xx = x + dx;
            zz += zz < 0 ? g.nz : (zz >= g.nz ? -g.nz : 0);
            yy += yy < 0 ? g.ny : (yy >= g.ny ? -g.ny : 0);
            xx += xx < 0 ? g.nx : (xx >= g.nx ? -g.nx : 0);
            if ((zz * g.ny + yy) * g.nx + xx < idx) { peak = false; break; }   // (equal: the cell itself, wrapped)
          }
      won |= peak ? (1u << lz) : 0u;
    }
#pragma unroll
    for (int lz = 0; lz < kVTileZ; ++lz)
      if (won & (1u << lz))
        mine[lz / 2] = cell_key(val[(lz + R) * HY * HX + lc], ((z0 + lz) * g.ny + y) * g.nx + x);
  }

  // keys after the volume's cutoff go first: the cutoff is the K-th key of
  // a tile that held at least K, all earlier, so none of them can be among
  // the volume's first K.  It only decreases, and every value it takes is
  // safe, so a stale read merely prunes less.
  const uint64_t cmax = __hip_atomic_load(cut, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
  for (int j = 0; j < NS; ++j) mine[j] = mine[j] > cmax ? kNoKey : mine[j];

  // the block's first K keys: gather every thread's keys in LDS (over the
  // staged values, which are no longer read; one atomic per wave and slot,
  // lanes placed by their rank among the wave's keys), sort the keys present
  // once, keep K and publish the K-th as the cutoff.  Fewer than K are
  // written unsorted (the reduction sorts).  The gather order varies from
  // run to run; the reduced lists do not.
  if (tid == 0) *nkeys = 0;
  __syncthreads();
  uint64_t* keys = reinterpret_cast<uint64_t*>(val);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const bool have = mine[j] != kNoKey;
    const uint64_t b = __ballot(have);
    if (b == 0) continue;   // uniform
    int base = 0;
    if (lane == 0) base = atomicAdd(nkeys, (int)__popcll(b));
    base = __shfl(base, 0, 64);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (have) keys[base + rank] = mine[j];
  }
  __syncthreads();
  const int n = *nkeys;
  if (n <= K) {
    for (int i = tid; i < K; i += kPeakThreads) dst[i] = i < n ? keys[i] : kNoKey;
  } else if (n <= 128) {   // the usual case: one wave sorts in registers
    if (wave == 0) {
      uint64_t a = lane < n ? keys[lane] : kNoKey, b = lane + 64 < n ? keys[lane + 64] : kNoKey;
      wave_sort128(a, b, lane);
      if (lane < K) dst[lane] = a;
      if (lane + 64 < K) dst[lane + 64] = b;
      const uint64_t src = K <= 64 ? a : b;   // n > K: the K-th key sits in lane (K - 1) mod 64
      const int kl = (K - 1) & 63;
      const uint64_t kth = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(src >> 32), kl) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)src, kl);
      if (lane == 0) atomicMin(reinterpret_cast<unsigned long long*>(cut), (unsigned long long)kth);
    }
  } else {
    int np = 1;
    while (np < n) np <<= 1;
    for (int i = n + tid; i < np; i += kPeakThreads) keys[i] = kNoKey;
    __syncthreads();
    bitonic_sort_n<kPeakThreads>(keys, np);
    for (int i = tid; i < K; i += kPeakThreads) dst[i] = keys[i];
    if (tid == 0) atomicMin(reinterpret_cast<unsigned long long*>(cut), (unsigned long long)keys[K - 1]);
  }
}

// One tile per block, any volume shape.  Output: one list of K keys per tile,
// [volume][tile][K].
template <int RADIUS>
__global__ void __launch_bounds__(kPeakThreads)
    k_vpeaks_tile(const float* __restrict__ params, VolGeom g, int tiles, int K, float thr_below, int wrap, int keep_border,
                  uint64_t* __restrict__ cut, uint64_t* __restrict__ out) {
  using T = VTile<RADIUS>;
  __shared__ __align__(16) float val[T::NH];
  __shared__ int nkeys;
  // consecutive tiles (x fastest, then y, then z) share halo rows: keep them on one XCD's L2
  const int logical = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const typename T::Origin o = T::origin(g, tiles, logical);
  const float* P = params + (long long)o.vol * g.stride;
  if (o.x0 + kVTileX <= g.nx && (g.nx & 3) == 0 && ((uintptr_t)P & 15) == 0) {
    typename T::Regs q;
    T::load_vec(P, g, o, wrap, q);
    T::store_vec(val, q);
  } else {
    T::stage_scalar(val, P, g, o, wrap);
  }
  __syncthreads();
  vtile_detect<RADIUS>(val, &nkeys, g, o, K, thr_below, keep_border, cut + o.vol,
                       out + ((long long)o.vol * tiles + o.tile) * K);
}

// One sorted list of K keys per volume -> plane records and counts.
__global__ void __launch_bounds__(kMergeThreads)
    k_vpeaks_records(const float* __restrict__ params, VolGeom g, int K, const uint64_t* __restrict__ list, int ns,
                     int sp, int space_id, ft_plane_peak* __restrict__ peaks, int32_t* __restrict__ n_found) {
  const int vol = blockIdx.x;
  const float* P = params + (long long)vol * g.stride;
  const uint64_t* keys = list + (long long)vol * K;
  ft_plane_peak* dst = peaks + ((long long)vol * ns + sp) * K;
  for (int i = threadIdx.x; i < K; i += kMergeThreads) {
    if (keys[i] == kNoKey) continue;
    const int idx = (int)(uint32_t)(keys[i] & 0xffffffffu);
    const int z = idx / (g.ny * g.nx), rem = idx % (g.ny * g.nx);
    const int r = rem / g.nx, c = rem % g.nx;
    ft_plane_peak pk;
    pk.volume = vol;
    pk.space = space_id;
    pk.z = z;
    pk.row = r;
    pk.col = c;
    pk.value = fabsf(P[idx]);
    pk.a = -2.0f * (float)(c - g.nx / 2) / (float)g.nx;
    pk.b = -2.0f * (float)(r - g.ny / 2) / (float)g.ny;
    pk.c = (float)(z - g.nz / 2) - pk.a * (float)(g.nx / 2) - pk.b * (float)(g.ny / 2) + (float)(g.zimg / 2);
    dst[i] = pk;
  }
  if (threadIdx.x == 0) {
    int count = 0;
    while (count < K && keys[count] != kNoKey) ++count;
    n_found[(long long)vol * ns + sp] = count;
  }
}

int vpeaks_tiles(int nz, int ny, int nx) {
  return ((nz + kVTileZ - 1) / kVTileZ) * ((ny + kVTileY - 1) / kVTileY) * ((nx + kVTileX - 1) / kVTileX);
}

// stage-1 lists (one per tile), then the first reduction level's lists, then
// one cutoff key per volume
size_t vpeaks_workspace_bytes(int nvol, int tiles, int K) {
  const size_t lvl1 = ((size_t)tiles + merge_group(K) - 1) / merge_group(K);
  return (size_t)nvol * (((size_t)tiles + lvl1) * (size_t)K + 1) * sizeof(uint64_t);
}

hipError_t launch_vpeaks(const float* params, long long stride, int batch, int nz, int ny, int nx, int zimg, int K,
                         float thr, int radius, int wrap, int keep_border, int ns, int sp, int space_id,
                         ft_plane_peak* peaks, int32_t* n_found, void* ws, hipStream_t s) {
  const VolGeom g{nz, ny, nx, zimg, stride};
  const int tiles = vpeaks_tiles(nz, ny, nx);
  if (radius < 1 || radius > 2) return hipErrorInvalidValue;
  const size_t lvl1 = ((size_t)tiles + merge_group(K) - 1) / merge_group(K);
  uint64_t* cand = static_cast<uint64_t*>(ws);
  uint64_t* cut = cand + (size_t)batch * ((size_t)tiles + lvl1) * K;   // as vpeaks_workspace_bytes lays it out
  k_fill_keys<<<(batch + 255) / 256, 256, 0, s>>>(cut, batch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid(tiles, batch);
  const float thr_below = std::nextafter(thr, -INFINITY);   // v >= thr  <=>  v > thr_below
  if (radius == 1)
    k_vpeaks_tile<1><<<grid, kPeakThreads, 0, s>>>(params, g, tiles, K, thr_below, wrap, keep_border, cut, cand);
  else
    k_vpeaks_tile<2><<<grid, kPeakThreads, 0, s>>>(params, g, tiles, K, thr_below, wrap, keep_border, cut, cand);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint64_t* list = nullptr;
  e = reduce_lists(cand, batch, tiles, K, cut, &list, s);
  if (e != hipSuccess) return e;
  k_vpeaks_records<<<batch, kMergeThreads, 0, s>>>(params, g, K, list, ns, sp, space_id, peaks, n_found);
  return hipGetLastError();
}

}  // namespace funnel
