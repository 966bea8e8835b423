// funnel_queue.hpp -- the work-queue schedule of ragged batches: one
// persistent launch per pass kind over (class, space, image, tile) items.
#pragma once

#include <hip/hip_runtime.h>

#include "funnel_internal.hpp"

// Transform lengths with queue kernels: (slot, length).  Column lengths are
// the padded lengths Np = N + M and row lengths the widths and heights of
// the camera formats 240x320, 480x640, 720x1280 and 1080x1920.
#define FUNNEL_QUEUE_COL_LENGTHS(X) X(0, 560) X(1, 1120) X(2, 2000) X(3, 3000)
#define FUNNEL_QUEUE_ROW_LENGTHS(X) X(0, 240) X(1, 320) X(2, 480) X(3, 640) X(4, 720) X(5, 1080) X(6, 1280) X(7, 1920)

namespace funnel {

constexpr int kQueueColThreads = 1024;  // block size of the column-pass queue kernels
constexpr int kQueueRowThreads = 256;   // and of the row-pass one
constexpr int kQueueSegs = 16;          // segments (class x space) per launch

// One segment of a launch's items: one size class in one space.  Its items
// are first .. first + count - 1, item first + img * tiles + tile.
struct QueueSeg {
  int kind;            // length slot: column length (R2C, C2R) or row length (rows)
  int trans;           // column passes: the lines are image rows
  int accum;           // C2R: add to the output; rows: the adjoint
  int first;           // first item of the segment
  int tiles;           // items per image: column tiles, or blocks of rows
  int nlines, a, b;    // R2C: lines, lin, off; C2R: lines, r0, nout; rows: a = Np, b = h
  float scale;
  long long stride;    // rows: complex values per image of the spectrum
  ImgMap map;          // column passes: where image i's input and output start
  const void* in;      // column passes: input base
  void* out;           // column passes: output base; rows: the spectrum (in place)
  const float2* tw;    // twiddles of the segment's length
};

struct QueueArgs {
  int nseg;
  int total;           // items of all segments
  int* counter;        // the queue: next item to take (0 at launch)
  QueueSeg seg[kQueueSegs];
};

enum class QueuePass { R2C, C2R, ROW };

// slot of a length, -1 when it has no queue kernel
int queue_col_kind(int L);
int queue_row_kind(int M);
// column tiles per image of a column pass at length L with `nlines` lines
// (shape 0: 16 elements per thread, 1: 32), rows per block of a row pass
int queue_col_tiles(int L, int shape, int nlines);
int queue_row_rows(int M);
// zero n queue counters (a kernel, so that graphs replay it)
hipError_t launch_queue_reset(int* counters, int n, hipStream_t s);
// blocks of the persistent grid of a queue kernel on the current device (as
// many as it keeps resident at once), queried once at plan creation
hipError_t queue_grid_size(QueuePass pass, int shape, int* grid);
// one persistent launch of `grid` blocks over q's items (shape: the column
// passes' tile shape, 0: 16 elements per thread, 1: 32)
hipError_t launch_queue(QueuePass pass, int shape, int grid, const QueueArgs& q, hipStream_t s);

}  // namespace funnel
