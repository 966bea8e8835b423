// funnel_queue.hip -- ragged batches in one persistent launch per pass kind.
//
// A ragged batch holds images of several sizes (size classes).  Instead of
// one launch per class and pass, each pass kind runs as ONE persistent
// launch over a device-side work queue: the grid holds as many blocks as the
// GPU keeps resident at once, and each block repeatedly takes the next item
// -- one column tile, or one block of frequency rows, of one image of one
// class and space -- from a counter in the caller's workspace (atomicAdd),
// until the queue is empty.  Every block reaches the exit once the counter
// has passed the last item.
//
// Items are numbered segment by segment (a segment is one class in one
// space; the host orders them longest transform first, so the largest items
// are taken first and the short ones fill the tail).  A block decodes its
// item to (segment, image, tile) and runs that length's tile function -- the
// same code the per-class kernels run (funnel_passes.hpp) -- with its own
// tile shape: the block size is fixed per launch, so each length takes as
// many column pairs (rows) as fit and the threads beyond its tile idle
// through the barriers.
//
// Lengths with queue kernels: the column lengths Np and row lengths of the
// camera formats 240x320, 480x640, 720x1280 and 1080x1920 (Np = N + M).
// A ragged plan whose classes all use these lengths may run this schedule.
#include "funnel_passes.hpp"
#include "funnel_queue.hpp"

namespace funnel {

// Tile shape of column length L in a block of T threads: E elements per
// thread (P = ceil(L / E) threads per transform), as many column pairs as
// the block's threads and 150 KB of LDS hold, at most 32.
constexpr int cmin(int a, int b) { return a < b ? a : b; }
template <int L, int E, int T>
struct QCol {
  static constexpr int P = FastCfg<L, E, 1, 1>::P;
  static constexpr int LINES = cmin(cmin(T / P, 32), (150 * 1024) / ((L + L / 16 + 1) * 4));
  using Cfg = FastCfg<L, E, LINES, 1>;
  static_assert(LINES >= 1 && Cfg::valid && Cfg::THREADS <= T, "queue tile must fit the block");
  static constexpr int lds_floats = LayInterR<LINES>::size(L);
};

// Row tile of row length M: the per-class kernels' 16-element, 256-thread tile.
template <int M>
struct QRow {
  using Cfg = RowFastCfg<M, 16, kQueueRowThreads>;
  static_assert(Cfg::valid && Cfg::THREADS <= kQueueRowThreads, "queue row tile must fit the block");
  static constexpr int lds_float2 = LayRow<Cfg::ROWS, M>::size(M);
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int E>
constexpr int col_lds_floats() {
  int m = 0;
#define FUNNEL_Q(k, L) m = cmax(m, QCol<L, E, kQueueColThreads>::lds_floats);
  FUNNEL_QUEUE_COL_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  return m;
}

constexpr int row_lds_float2() {
  int m = 0;
#define FUNNEL_Q(k, M) m = cmax(m, QRow<M>::lds_float2);
  FUNNEL_QUEUE_ROW_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  return m;
}

// Take the next item: one thread draws it, the block reads it from LDS.
// The second barrier keeps the draw of the next item behind every read.
__device__ __forceinline__ int queue_next(int* counter, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  const int item = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();
  return item;
}

// The thread index through an empty asm, once per item: nothing a tile
// function derives from it (addresses of every case of the switch) is then
// hoisted out of the item loop and kept live across all items.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// the segment holding `item` (segments are few; `item` is block-uniform)
__device__ __forceinline__ int queue_segment(const QueueArgs& q, int item) {
  int s = 0;
  while (s + 1 < q.nseg && item >= q.seg[s + 1].first) ++s;
  return s;
}

// R2C column pass (pass A of the forward, pass C^T of the adjoint)
template <int E>
__global__ void __launch_bounds__(kQueueColThreads) k_queue_r2c(QueueArgs q) {
  __shared__ float lds[col_lds_floats<E>()];
  __shared__ int slot;
  for (;;) {
    const int item = queue_next(q.counter, &slot);
    if (item >= q.total) break;
    const QueueSeg& g = q.seg[queue_segment(q, item)];
    const int local = item - g.first, tile = local % g.tiles, img = local / g.tiles;
    const int tid = opaque_tid();
    const float* in = static_cast<const float*>(g.in);
    float2* out = static_cast<float2*>(g.out);
    switch (g.kind * 2 + g.trans) {
#define FUNNEL_Q(k, L)                                                                                         \
  case 2 * k:                                                                                                  \
    r2c_tile<L, E, QCol<L, E, kQueueColThreads>::LINES, 1, false, kPrecFP32>(                                  \
        in, out, g.nlines, g.a, g.b, g.map, g.scale, g.tw, tile, img, tid,                                     \
        tid < QCol<L, E, kQueueColThreads>::Cfg::THREADS, lds);                                        \
    break;                                                                                                     \
  case 2 * k + 1:                                                                                              \
    r2c_tile<L, E, QCol<L, E, kQueueColThreads>::LINES, 1, true, kPrecFP32>(                                   \
        in, out, g.nlines, g.a, g.b, g.map, g.scale, g.tw, tile, img, tid,                                     \
        tid < QCol<L, E, kQueueColThreads>::Cfg::THREADS, lds);                                        \
    break;
      FUNNEL_QUEUE_COL_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
      default: break;
    }
  }
}

// C2R column pass (pass C of the forward, pass A^T of the adjoint: the
// inverse space writes the image gradient transposed, the regular space
// then adds its columns)
template <int E>
__global__ void __launch_bounds__(kQueueColThreads) k_queue_c2r(QueueArgs q) {
  __shared__ float lds[col_lds_floats<E>()];
  __shared__ int slot;
  for (;;) {
    const int item = queue_next(q.counter, &slot);
    if (item >= q.total) break;
    const QueueSeg& g = q.seg[queue_segment(q, item)];
    const int local = item - g.first, tile = local % g.tiles, img = local / g.tiles;
    const int tid = opaque_tid();
    const float2* in = static_cast<const float2*>(g.in);
    float* out = static_cast<float*>(g.out);
    switch (g.kind * 4 + g.trans * 2 + g.accum) {
#define FUNNEL_Q(k, L)                                                                                         \
  case 4 * k:                                                                                                  \
    c2r_tile<L, E, QCol<L, E, kQueueColThreads>::LINES, 1, false, false, kPrecFP32>(                           \
        in, out, g.nlines, g.a, g.b, g.map, g.scale, g.tw, tile, img, tid,                                     \
        tid < QCol<L, E, kQueueColThreads>::Cfg::THREADS, lds);                                        \
    break;                                                                                                     \
  case 4 * k + 1:                                                                                              \
    c2r_tile<L, E, QCol<L, E, kQueueColThreads>::LINES, 1, false, true, kPrecFP32>(                            \
        in, out, g.nlines, g.a, g.b, g.map, g.scale, g.tw, tile, img, tid,                                     \
        tid < QCol<L, E, kQueueColThreads>::Cfg::THREADS, lds);                                        \
    break;                                                                                                     \
  case 4 * k + 2:                                                                                              \
    c2r_tile<L, E, QCol<L, E, kQueueColThreads>::LINES, 1, true, false, kPrecFP32>(                            \
        in, out, g.nlines, g.a, g.b, g.map, g.scale, g.tw, tile, img, tid,                                     \
        tid < QCol<L, E, kQueueColThreads>::Cfg::THREADS, lds);                                        \
    break;
      FUNNEL_QUEUE_COL_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
      default: break;
    }
  }
}

// Row pass: NVMT + DFT along x' (forward) or its transpose (adjoint), in place.
__global__ void __launch_bounds__(kQueueRowThreads) k_queue_row(QueueArgs q) {
  __shared__ float2 lds[row_lds_float2()];
  __shared__ int slot;
  for (;;) {
    const int item = queue_next(q.counter, &slot);
    if (item >= q.total) break;
    const QueueSeg& g = q.seg[queue_segment(q, item)];
    const int local = item - g.first, blk = local % g.tiles, img = local / g.tiles;
    const int tid = opaque_tid();
    float2* data = static_cast<float2*>(g.out);
    switch (g.kind * 2 + g.accum) {   // accum: the adjoint
#define FUNNEL_Q(k, M)                                                                                         \
  case 2 * k:                                                                                                  \
    row_tile<M, 16, kQueueRowThreads, false, kPrecFP32>(data, g.a, g.b, 1, g.stride, g.tw, blk, img,           \
                                                        tid, tid < QRow<M>::Cfg::THREADS, lds);                 \
    break;                                                                                                     \
  case 2 * k + 1:                                                                                              \
    row_tile<M, 16, kQueueRowThreads, true, kPrecFP32>(data, g.a, g.b, 1, g.stride, g.tw, blk, img,            \
                                                       tid, tid < QRow<M>::Cfg::THREADS, lds);                  \
    break;
      FUNNEL_QUEUE_ROW_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
      default: break;
    }
  }
}

__global__ void k_queue_reset(int* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counters[i] = 0;
}

int queue_col_kind(int L) {
  switch (L) {
#define FUNNEL_Q(k, n) case n: return k;
    FUNNEL_QUEUE_COL_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  }
  return -1;
}

int queue_row_kind(int M) {
  switch (M) {
#define FUNNEL_Q(k, n) case n: return k;
    FUNNEL_QUEUE_ROW_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  }
  return -1;
}

int queue_col_tiles(int L, int shape, int nlines) {
  const int pairs = nlines / 2;
  switch (L) {
#define FUNNEL_Q(k, n)                                                                                         \
  case n: {                                                                                                    \
    const int lines = shape == 0 ? QCol<n, 16, kQueueColThreads>::LINES : QCol<n, 32, kQueueColThreads>::LINES; \
    return (pairs + lines - 1) / lines;                                                                        \
  }
    FUNNEL_QUEUE_COL_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  }
  return 0;
}

int queue_row_rows(int M) {
  switch (M) {
#define FUNNEL_Q(k, n) case n: return QRow<n>::Cfg::ROWS;
    FUNNEL_QUEUE_ROW_LENGTHS(FUNNEL_Q)
#undef FUNNEL_Q
  }
  return 0;
}

namespace {
template <class Kern>
hipError_t resident_blocks(Kern kern, int threads, int* grid) {
  int dev = 0, cus = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kern), threads, 0);
  if (e != hipSuccess) return e;
  *grid = cus * (occ > 0 ? occ : 1);
  return hipSuccess;
}
}  // namespace

hipError_t queue_grid_size(QueuePass pass, int shape, int* grid) {
  switch (pass) {
    case QueuePass::R2C: return shape == 0 ? resident_blocks(k_queue_r2c<16>, kQueueColThreads, grid)
                                           : resident_blocks(k_queue_r2c<32>, kQueueColThreads, grid);
    case QueuePass::C2R: return shape == 0 ? resident_blocks(k_queue_c2r<16>, kQueueColThreads, grid)
                                           : resident_blocks(k_queue_c2r<32>, kQueueColThreads, grid);
    case QueuePass::ROW: return resident_blocks(k_queue_row, kQueueRowThreads, grid);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_queue_reset(int* counters, int n, hipStream_t s) {
  k_queue_reset<<<1, 64, 0, s>>>(counters, n);
  return hipGetLastError();
}

hipError_t launch_queue(QueuePass pass, int shape, int grid, const QueueArgs& q, hipStream_t s) {
  if (q.total <= 0) return hipSuccess;
  if (q.nseg < 1 || q.nseg > kQueueSegs || shape < 0 || shape > 1 || grid < 1) return hipErrorInvalidValue;
  if (grid > q.total) grid = q.total;
  switch (pass) {
    case QueuePass::R2C:
      if (shape == 0) k_queue_r2c<16><<<grid, kQueueColThreads, 0, s>>>(q);
      else k_queue_r2c<32><<<grid, kQueueColThreads, 0, s>>>(q);
      break;
    case QueuePass::C2R:
      if (shape == 0) k_queue_c2r<16><<<grid, kQueueColThreads, 0, s>>>(q);
      else k_queue_c2r<32><<<grid, kQueueColThreads, 0, s>>>(q);
      break;
    case QueuePass::ROW: k_queue_row<<<grid, kQueueRowThreads, 0, s>>>(q); break;
  }
  return hipGetLastError();
}

}  // namespace funnel
