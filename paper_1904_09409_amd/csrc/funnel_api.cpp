// funnel_api.cpp -- the C ABI declared in include/funnel.h: argument
// validation (host only, before any device work), plans with their FP64-derived
// twiddle tables, workspace layout, the order of the passes, ragged batches,
// graphs, autotuning and kernel timing.
//
// A plan is a list of size classes.  A uniform batch is one class with
// uniform strides; a ragged batch groups its images by (rows, cols), each
// class with its own radix schedule, tile variants, twiddles, workspace region
// and device tables of per-image offsets.  The classes of a ragged plan run on
// their own streams (default priority), forked from and joined back to the
// caller's stream by events, so they overlap on the device -- eagerly or
// inside a captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/funnel.h"
#include "fft_mfma.hpp"   // (the matrix-core passes' radix plan, for their twiddle tables)
#include "funnel_internal.hpp"
#include "funnel_queue.hpp"

// Event pairs around each launch, filled while profiling is enabled.
struct FtProfiler {
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<std::string> name;
  std::vector<double> bytes;
};

// The twelve kernel launches of a class: three passes per space, forward and adjoint.
enum Role { FA_REG, FB_REG, FC_REG, FA_INV, FB_INV, FC_INV, AC_REG, AB_REG, AA_REG, AC_INV, AB_INV, AA_INV, NROLES };
static const char* const kRoleName[NROLES] = {
    "fwd.regular.A", "fwd.regular.B", "fwd.regular.C", "fwd.inverse.A", "fwd.inverse.B", "fwd.inverse.C",
    "adj.regular.Ct", "adj.regular.Bt", "adj.regular.At", "adj.inverse.Ct", "adj.inverse.Bt", "adj.inverse.At"};

// The launches of the queue schedule: forward A, B, C; adjoint C^T, B^T, and
// A^T in two launches (the inverse space writes dI, the regular space then
// adds to it).  Each has its own counter in the workspace.
enum QLaunch { QF_A, QF_B, QF_C, QA_CT, QA_BT, QA_AT_INV, QA_AT_REG, kQueueLaunches };
static const char* const kQueueName[kQueueLaunches] = {"queue.fwd.A", "queue.fwd.B", "queue.fwd.C",
                                                       "queue.adj.Ct", "queue.adj.Bt", "queue.adj.At.inverse",
                                                       "queue.adj.At.regular"};

struct FtClass {
  int N = 0, M = 0, Np = 0, h = 0, count = 0;
  size_t tw_np = 0, tw_m = 0, tw_n = 0;   // float2 offsets of this class's tables in plan->tw
  size_t tw_2m = 0, tw_2n = 0;            // chirp-z plans: twiddles of the length-2W transforms
  size_t cz_m = 0, wz_m = 0, cz_n = 0, wz_n = 0;   // chirp-z plans: float2 offsets in plan->chirp
  size_t ws_reg = 0, ws_inv = 0;          // byte offsets of the half spectra in the workspace
  size_t off_inv_plane = 0;               // floats from an image's plane block to its inverse plane
  long long img_stride = 0, plane_stride = 0;
  const long long* d_img_off = nullptr;   // ragged: class-local image -> element offset
  const long long* d_plane_off = nullptr;
  const int* d_gidx = nullptr;            // ragged: class-local image -> caller's image index
  std::vector<int> images;                // caller's image indices (host copy)
  int variant[NROLES] = {};
  hipStream_t stream = nullptr;           // ragged plans with several classes
  hipEvent_t done = nullptr;
};

struct ft_plan {
  FtProfiler* prof = nullptr;
  int device = 0;
  int spaces = 0;
  int batch = 0;
  int prec = 0;             // FT_PREC_*
  bool chirpz = false;      // FT_PLAN_NVMT_CHIRPZ: band-limited NVMT in the row passes
  bool ragged = false;
  // ragged plans: FT_SCHEDULE_CLASS_STREAMS (each size class's launches on a
  // stream of its own) or FT_SCHEDULE_QUEUE (one persistent launch per pass
  // kind over all classes, funnel_queue.hip), the latter only where every
  // class's lengths have queue kernels (queue_ok)
  int schedule = FT_SCHEDULE_CLASS_STREAMS;
  bool queue_ok = false;
  int qshape[kQueueLaunches] = {};  // tile shape of each queue launch (column passes: 0 or 1)
  int qgrid[3][2] = {};             // persistent grid of each queue kernel (pass, shape)
  size_t ws_queue = 0;              // byte offset of the queue counters in the workspace
  std::vector<FtClass> cls;
  float2* tw = nullptr;
  float2* chirp = nullptr;  // chirp-z plans: per-row chirp spectra and chirps
  void* tables = nullptr;
  size_t ws_bytes = 0;
  size_t plane_elems = 0;   // uniform: floats per image; ragged: extent of the whole planes buffer
  size_t image_extent = 0;  // floats of the images buffer
  size_t plane_extent = 0;  // floats of the planes buffer
  hipEvent_t fork = nullptr;
};

struct ft_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

namespace {

thread_local std::string g_err;

ft_status fail(ft_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

ft_status ok() {
  g_err.clear();
  return FT_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

ft_status check_device(const ft_plan* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FT_ERR_NO_DEVICE, "no HIP device");
  if (dev != p->device) return fail(FT_ERR_NO_DEVICE, "plan was created on device %d, current is %d", p->device, dev);
  return FT_OK;
}

ft_status hip_fail(hipError_t e, const char* what) {
  return fail(FT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// ------------------------------------------------------------------ static peak scratch
//
// funnel_peaks_noalloc keeps the partial peak lists and per-plane cutoffs in
// this array instead of a caller workspace.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the name stands
// for a host-side shadow, not a device address: host code uses only the
// address hipGetSymbolAddress returns for each device, resolved once per
// device (with that device current) when a plan is created there.
constexpr size_t kPeakScratchBytes = FT_PEAKS_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kPeakScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxScratchDevices] = {};

// The device address of `scratch` on device dev (the current device when it
// is first resolved).
ft_status scratch_for_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(FT_ERR_NO_DEVICE, "device %d is beyond the %d the peak scratch table covers", dev, kMaxScratchDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch[dev];
  return FT_OK;
}

// exp(-i 2 pi m / L), m = 0 .. L-1, evaluated in double and rounded to float
void fill_twiddles(float2* dst, int L) {
  for (int m = 0; m < L; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)L;
    dst[m] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
}

// The matrix-core passes' lane tables behind the length-L table (entries
// exp(-i 2 pi e / L) for the exponents the layout of mfma_lane_twiddle_offset
// names, evaluated in double as fill_twiddles does).
void fill_mfma_lane_twiddles(float2* dst, int L) {
  const funnel::RadixPlan pl = funnel::mfma_plan(L);
  int ns = pl.n > 0 ? pl.r[0] : 1;
  for (int I = 1; I < pl.n; ++I) {
    const int R = pl.r[I], per = R / 4;
    float2* t = dst + funnel::mfma_lane_twiddle_offset(L, I);
    for (int m = 0; m < ns; ++m)
      for (int g = 0; g < 4; ++g)
        for (int i = 0; i < per; ++i) {
          const long long e = (long long)(g * per + i) * m * (L / (ns * R));
          const double a = 2.0 * M_PI * (double)e / (double)L;
          t[(m * 4 + g) * per + i] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
        }
    ns *= R;
  }
}

bool role_is_row(int r) { return r == FB_REG || r == FB_INV || r == AB_REG || r == AB_INV; }
bool role_regular(int r) { return r <= FC_REG || (r >= AC_REG && r <= AA_REG); }
bool role_active(const ft_plan* p, int r) {
  return (p->spaces & (role_regular(r) ? FT_SPACE_REGULAR : FT_SPACE_INVERSE)) != 0;
}
unsigned role_mask(const ft_plan* p, const FtClass& c, int r) {
  if (!role_is_row(r)) return funnel::col_variant_mask(c.Np, p->prec);
  const int W = role_regular(r) ? c.M : c.N;
  return p->chirpz ? funnel::chirp_variant_mask(W) : funnel::row_variant_mask(W, p->prec);
}

// Algorithmic HBM bytes of one launch: each input read once, each output
// written once (a read-modify-write output counts twice).
double role_bytes(const ft_plan* p, const FtClass& c, int r) {
  const double B = c.count, N = c.N, M = c.M, Np = c.Np, h = c.h;
  const double W = role_regular(r) ? M : N;  // lines of the spectrum
  switch (r) {
    case FA_REG: case FA_INV: return B * (4.0 * N * M + 8.0 * h * W);
    // chirp-z rows also read the row's chirp spectrum (2W) and chirp (W) once
    case FB_REG: case FB_INV: case AB_REG: case AB_INV: return B * 16.0 * h * W + (p->chirpz ? 24.0 * h * W : 0.0);
    case FC_REG: case FC_INV: return B * (8.0 * h * W + 4.0 * Np * W);
    case AC_REG: case AC_INV: return B * (4.0 * Np * W + 8.0 * h * W);
    case AA_REG: return B * (8.0 * h * M + ((p->spaces & FT_SPACE_INVERSE) ? 8.0 : 4.0) * N * M);
    case AA_INV: return B * (8.0 * h * N + 4.0 * N * M);
  }
  return 0.0;
}

// Run one launch, bracketed by events when the plan is being profiled.
template <class Plan, class Fn>
hipError_t timed(const Plan* p, hipStream_t s, const std::string& name, double bytes, Fn&& fn) {
  FtProfiler* pr = p->prof;
  if (!pr || pr->used >= pr->cap) return fn();
  const int i = pr->used++;
  hipError_t e = hipEventRecord(pr->ev0[i], s);
  if (e != hipSuccess) return e;
  e = fn();
  if (e != hipSuccess) return e;
  pr->name[i] = name;
  pr->bytes[i] = bytes;
  return hipEventRecord(pr->ev1[i], s);
}

void free_profiler(FtProfiler* pr) {
  if (!pr) return;
  for (auto ev : pr->ev0) (void)hipEventDestroy(ev);
  for (auto ev : pr->ev1) (void)hipEventDestroy(ev);
  delete pr;
}

void free_plan(ft_plan* p) {
  if (!p) return;
  free_profiler(p->prof);
  for (auto& c : p->cls) {
    if (c.stream) (void)hipStreamDestroy(c.stream);
    if (c.done) (void)hipEventDestroy(c.done);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->tw) (void)hipFree(p->tw);
  if (p->chirp) (void)hipFree(p->chirp);
  if (p->tables) (void)hipFree(p->tables);
  delete p;
}

// One pass launch of class c.  src: images (forward) or plane gradients
// (adjoint); dst: planes (forward) or image gradients (adjoint).
hipError_t run_role(const ft_plan* p, const FtClass& c, int r, int v, const float* src, float* dst, char* w,
                    hipStream_t s) {
  const int B = c.count, N = c.N, M = c.M, Np = c.Np, h = c.h;
  const float2* tw_np = p->tw + c.tw_np;
  float2* Sr = reinterpret_cast<float2*>(w + c.ws_reg);
  float2* Si = reinterpret_cast<float2*>(w + c.ws_inv);
  const long long sr = (long long)h * M, si = (long long)h * N;
  const bool inv = p->spaces & FT_SPACE_INVERSE;
  using funnel::ImgMap;
  // where each launch's input and output of image i start
  const ImgMap img_to_sr{c.img_stride, sr, c.d_img_off, nullptr};
  const ImgMap img_to_si{c.img_stride, si, c.d_img_off, nullptr};
  const ImgMap sr_to_pl{sr, c.plane_stride, nullptr, c.d_plane_off};
  const ImgMap si_to_pl{si, c.plane_stride, nullptr, c.d_plane_off};
  const ImgMap pl_to_sr{c.plane_stride, sr, c.d_plane_off, nullptr};
  const ImgMap pl_to_si{c.plane_stride, si, c.d_plane_off, nullptr};
  const ImgMap sr_to_img{sr, c.img_stride, nullptr, c.d_img_off};
  const ImgMap si_to_img{si, c.img_stride, nullptr, c.d_img_off};
  switch (r) {
    // forward, regular space: y DFT of the image columns on the expanded frame,
    // NVMT + x' DFT per frequency row, Hermitian inverse y DFT
    case FA_REG: return funnel::launch_r2c(Np, v, p->prec, false, src, Sr, M, N, (Np - N) / 2, img_to_sr, 1.0f, tw_np, B, s);
    case FB_REG:
      if (p->chirpz)
        return funnel::launch_chirp(M, v, false, Sr, h, sr, p->chirp + c.cz_m, p->chirp + c.wz_m, p->tw + c.tw_2m, B, s);
      return funnel::launch_row(M, v, p->prec, false, Sr, Np, h, 1, sr, p->tw + c.tw_m, B, s);
    case FC_REG:
      return funnel::launch_c2r(Np, v, p->prec, false, false, Sr, dst, M, 0, Np, sr_to_pl, 1.0f / Np, tw_np, B, s);
    // forward, inverse space: the same on the transposed image (rows read directly)
    case FA_INV: return funnel::launch_r2c(Np, v, p->prec, true, src, Si, N, M, (Np - M) / 2, img_to_si, 1.0f, tw_np, B, s);
    case FB_INV:
      if (p->chirpz)
        return funnel::launch_chirp(N, v, false, Si, h, si, p->chirp + c.cz_n, p->chirp + c.wz_n, p->tw + c.tw_2n, B, s);
      return funnel::launch_row(N, v, p->prec, false, Si, Np, h, 1, si, p->tw + c.tw_n, B, s);
    case FC_INV:
      return funnel::launch_c2r(Np, v, p->prec, false, false, Si, dst + c.off_inv_plane, N, 0, Np, si_to_pl, 1.0f / Np,
                                tw_np, B, s);
    // adjoint, regular space: (2/Np) y DFT of the plane columns, conjugate x'
    // DFT + transposed interpolation, real part of the conjugate y DFT cropped
    case AC_REG: return funnel::launch_r2c(Np, v, p->prec, false, src, Sr, M, Np, 0, pl_to_sr, 2.0f / Np, tw_np, B, s);
    case AB_REG:
      if (p->chirpz)
        return funnel::launch_chirp(M, v, true, Sr, h, sr, p->chirp + c.cz_m, p->chirp + c.wz_m, p->tw + c.tw_2m, B, s);
      return funnel::launch_row(M, v, p->prec, true, Sr, Np, h, 1, sr, p->tw + c.tw_m, B, s);
    // (the inverse space runs first; the regular space's columns add to its result)
    case AA_REG:
      return funnel::launch_c2r(Np, v, p->prec, false, inv, Sr, dst, M, (Np - N) / 2, N, sr_to_img, 0.5f, tw_np, B,
                                s);
    // adjoint, inverse space: transposed write into the image rows
    case AC_INV:
      return funnel::launch_r2c(Np, v, p->prec, false, src + c.off_inv_plane, Si, N, Np, 0, pl_to_si, 2.0f / Np, tw_np, B,
                                s);
    case AB_INV:
      if (p->chirpz)
        return funnel::launch_chirp(N, v, true, Si, h, si, p->chirp + c.cz_n, p->chirp + c.wz_n, p->tw + c.tw_2n, B, s);
      return funnel::launch_row(N, v, p->prec, true, Si, Np, h, 1, si, p->tw + c.tw_n, B, s);
    case AA_INV:
      return funnel::launch_c2r(Np, v, p->prec, true, false, Si, dst, N, (Np - M) / 2, M, si_to_img, 0.5f, tw_np, B,
                                s);
  }
  return hipErrorInvalidValue;
}

std::string role_label(const ft_plan* p, int ci, int r) {
  if (p->cls.size() == 1) return kRoleName[r];
  return "c" + std::to_string(ci) + "." + kRoleName[r];
}

// Launch order: forward A, B, C of the regular then the inverse space; the
// adjoint runs the inverse space first (its transposed pass writes dI) and the
// regular space's column pass adds to it (a read-modify-write of dI's columns
// is cheaper than one of its rows).
static const int kForwardOrder[] = {FA_REG, FB_REG, FC_REG, FA_INV, FB_INV, FC_INV};
static const int kAdjointOrder[] = {AC_INV, AB_INV, AA_INV, AC_REG, AB_REG, AA_REG};

// The queue schedule of a ragged plan: the forward as three persistent
// launches (A, B, C), the adjoint as four (C^T, B^T, inverse A^T, regular
// A^T), each over the items of every class and space, longest transforms
// first.  A fill kernel zeroes the direction's counters first (in the
// workspace, so concurrent calls with separate workspaces do not share them).
hipError_t enqueue_queue(const ft_plan* p, bool fwd, const float* src, float* dst, char* w, hipStream_t s) {
  using funnel::ImgMap;
  using funnel::QueueArgs;
  using funnel::QueueSeg;
  int* counters = reinterpret_cast<int*>(w + p->ws_queue);
  std::vector<int> order(p->cls.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return p->cls[a].Np > p->cls[b].Np; });
  const bool reg = p->spaces & FT_SPACE_REGULAR, inv = p->spaces & FT_SPACE_INVERSE;

  // segment of class c in one space for queue launch ql
  auto segment = [&](int ql, const FtClass& c, bool regular, int first, QueueSeg& g) {
    const int Np = c.Np, h = c.h, M = c.M, N = c.N;
    const int W = regular ? M : N;                       // lines of the spectrum
    float2* S = reinterpret_cast<float2*>(w + (regular ? c.ws_reg : c.ws_inv));
    const long long ss = (long long)h * W;
    const size_t plane_off = regular ? 0 : c.off_inv_plane;
    std::memset(&g, 0, sizeof g);
    g.first = first;
    g.tw = p->tw + c.tw_np;
    g.kind = funnel::queue_col_kind(Np);
    const int shape = p->qshape[ql];
    switch (ql) {
      case QF_A:   // image lines -> S (the inverse space reads image rows)
        g.trans = regular ? 0 : 1;
        g.nlines = W; g.a = regular ? N : M; g.b = (Np - (regular ? N : M)) / 2; g.scale = 1.0f;
        g.map = ImgMap{c.img_stride, ss, c.d_img_off, nullptr};
        g.in = src; g.out = S;
        g.tiles = funnel::queue_col_tiles(Np, shape, W);
        break;
      case QF_B: case QA_BT:   // rows of S in place
        g.kind = funnel::queue_row_kind(W);
        g.accum = ql == QA_BT;
        g.a = Np; g.b = h; g.stride = ss;
        g.out = S;
        g.tw = p->tw + (regular ? c.tw_m : c.tw_n);
        g.tiles = (h + funnel::queue_row_rows(W) - 1) / funnel::queue_row_rows(W);
        break;
      case QF_C:   // S -> plane columns, 1/Np
        g.nlines = W; g.a = 0; g.b = Np; g.scale = 1.0f / Np;
        g.map = ImgMap{ss, c.plane_stride, nullptr, c.d_plane_off};
        g.in = S; g.out = dst + plane_off;
        g.tiles = funnel::queue_col_tiles(Np, shape, W);
        break;
      case QA_CT:   // plane columns -> S, 2/Np
        g.nlines = W; g.a = Np; g.b = 0; g.scale = 2.0f / Np;
        g.map = ImgMap{c.plane_stride, ss, c.d_plane_off, nullptr};
        g.in = src + plane_off; g.out = S;
        g.tiles = funnel::queue_col_tiles(Np, shape, W);
        break;
      case QA_AT_INV: case QA_AT_REG:   // S -> image gradient (inverse: rows, written; regular: columns, added)
        g.trans = regular ? 0 : 1;
        g.accum = regular && inv;
        g.nlines = W; g.a = (Np - (regular ? N : M)) / 2; g.b = regular ? N : M; g.scale = 0.5f;
        g.map = ImgMap{ss, c.img_stride, nullptr, c.d_img_off};
        g.in = S; g.out = dst;
        g.tiles = funnel::queue_col_tiles(Np, shape, W);
        break;
    }
    return g.tiles * c.count;
  };

  const int first_ql = fwd ? QF_A : QA_CT, last_ql = fwd ? QF_C : QA_AT_REG;
  hipError_t e = funnel::launch_queue_reset(counters + first_ql, last_ql - first_ql + 1, s);
  for (int ql = first_ql; ql <= last_ql && e == hipSuccess; ++ql) {
    QueueArgs q;
    std::memset(&q, 0, sizeof q);
    q.counter = counters + ql;
    double bytes = 0.0;
    for (int ci : order) {
      const FtClass& c = p->cls[ci];
      for (int sp = 0; sp < 2; ++sp) {
        const bool regular = sp == 0;
        if (!(regular ? reg : inv)) continue;
        if (ql == QA_AT_INV && regular) continue;
        if (ql == QA_AT_REG && !regular) continue;
        q.total += segment(ql, c, regular, q.total, q.seg[q.nseg]);
        ++q.nseg;
      }
      static const int kRole[kQueueLaunches][2] = {{FA_REG, FA_INV}, {FB_REG, FB_INV}, {FC_REG, FC_INV},
                                                   {AC_REG, AC_INV}, {AB_REG, AB_INV}, {-1, AA_INV}, {AA_REG, -1}};
      for (int sp = 0; sp < 2; ++sp)
        if (kRole[ql][sp] >= 0 && role_active(p, kRole[ql][sp])) bytes += role_bytes(p, c, kRole[ql][sp]);
    }
    if (q.nseg == 0) continue;
    const funnel::QueuePass pass = (ql == QF_B || ql == QA_BT) ? funnel::QueuePass::ROW
                                   : (ql == QF_A || ql == QA_CT) ? funnel::QueuePass::R2C
                                                                 : funnel::QueuePass::C2R;
    const int shape = pass == funnel::QueuePass::ROW ? 0 : p->qshape[ql];
    const int grid = p->qgrid[(int)pass][shape];
    e = timed(p, s, kQueueName[ql], bytes, [&] { return funnel::launch_queue(pass, shape, grid, q, s); });
  }
  return e;
}

// Enqueue the roles of `order` for every class: on the caller's stream for a
// single class, else on the class streams between a fork and a join (or, for
// the queue schedule, as its persistent launches).
hipError_t enqueue_roles(const ft_plan* p, const int* order, const float* src, float* dst, char* w,
                         hipStream_t s) {
  if (p->schedule == FT_SCHEDULE_QUEUE) return enqueue_queue(p, order == kForwardOrder, src, dst, w, s);
  const bool fork = p->cls.size() > 1;
  hipError_t e = hipSuccess;
  if (fork) e = hipEventRecord(p->fork, s);
  for (size_t ci = 0; ci < p->cls.size() && e == hipSuccess; ++ci) {
    const FtClass& c = p->cls[ci];
    hipStream_t cs = fork ? c.stream : s;
    if (fork) e = hipStreamWaitEvent(cs, p->fork, 0);
    for (int i = 0; i < 6 && e == hipSuccess; ++i) {
      const int r = order[i];
      if (!role_active(p, r)) continue;
      e = timed(p, cs, role_label(p, (int)ci, r), role_bytes(p, c, r),
                [&] { return run_role(p, c, r, c.variant[r], src, dst, w, cs); });
    }
    if (fork && e == hipSuccess) e = hipEventRecord(c.done, cs);
  }
  for (size_t ci = 0; fork && ci < p->cls.size() && e == hipSuccess; ++ci)
    e = hipStreamWaitEvent(s, p->cls[ci].done, 0);
  return e;
}

ft_status check_call(const ft_plan* p, const void* a, const void* b, const void* ws, size_t ws_bytes) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!a || !b || !ws) return fail(FT_ERR_INVALID_ARG, "input, output and workspace must be non-NULL");
  if (!aligned16(a) || !aligned16(b) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  if (ws_bytes < p->ws_bytes)
    return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, p->ws_bytes);
  return FT_OK;
}

ft_status validate_shape(int N, int M, int spaces, long long Np) {
  if (N < 4 || M < 4 || (N & 1) || (M & 1))
    return fail(FT_ERR_INVALID_ARG, "rows and cols must be even and >= 4 (got %d x %d)", N, M);
  if (Np > (1 << 20) || M > (1 << 20) || N > (1 << 20))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "transform length too large");
  if (!funnel::length_supported((int)Np))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for padded length %lld", Np);
  if ((spaces & FT_SPACE_REGULAR) && !funnel::length_supported(M))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for row length %d (image width)", M);
  if ((spaces & FT_SPACE_INVERSE) && !funnel::length_supported(N))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for row length %d (image height)", N);
  // the kernels address one image's image, plane and spectrum blocks with
  // 32-bit byte offsets
  if (Np * (long long)(M > N ? M : N) * 8 >= (1ll << 31))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "per-image planes of %lld x %d exceed 2 GiB", Np, M > N ? M : N);
  return FT_OK;
}

size_t class_plane_floats(int spaces, const FtClass& c) {
  return ((spaces & FT_SPACE_REGULAR) ? (size_t)c.Np * c.M : 0) +
         ((spaces & FT_SPACE_INVERSE) ? (size_t)c.Np * c.N : 0);
}

// Shared tail of plan creation: geometry per class, workspace layout, default
// variants, twiddles, device tables, streams.  offsets: for ragged plans, per
// class the (image offset, plane offset) of each image; empty for uniform.
ft_status finish_plan(ft_plan* p, const std::vector<std::vector<std::pair<long long, long long>>>& offsets) {
  size_t ws = 0, ntw = 0;
  for (auto& c : p->cls) {
    c.h = c.Np / 2 - 1;
    c.off_inv_plane = (p->spaces & FT_SPACE_REGULAR) ? (size_t)c.Np * c.M : 0;
    c.ws_reg = ws;
    if (p->spaces & FT_SPACE_REGULAR) ws += align_up((size_t)c.count * c.h * c.M * sizeof(float2), 256);
    c.ws_inv = ws;
    if (p->spaces & FT_SPACE_INVERSE) ws += align_up((size_t)c.count * c.h * c.N * sizeof(float2), 256);
    // (split-precision plans: each table followed by the matrix-core lane tables)
    const bool lane = p->prec != FT_PREC_FP32;
    c.tw_np = ntw;
    ntw += c.Np + (lane ? funnel::mfma_lane_twiddles(c.Np) : 0);
    c.tw_m = ntw;
    ntw += c.M + (lane ? funnel::mfma_lane_twiddles(c.M) : 0);
    c.tw_n = ntw;
    ntw += c.N + (lane ? funnel::mfma_lane_twiddles(c.N) : 0);
    if (p->chirpz) {
      c.tw_2m = ntw;
      ntw += 2 * (size_t)c.M;
      c.tw_2n = ntw;
      ntw += 2 * (size_t)c.N;
    }
    for (int r = 0; r < NROLES; ++r) {
      const unsigned m = role_mask(p, c, r);
      c.variant[r] = 0;
      for (int v = 0; v < funnel::kMaxVariants; ++v)
        if (m & (1u << v)) {
          c.variant[r] = v;
          break;
        }
    }
  }
  if (!offsets.empty()) {
    // the queue schedule's counters, one 4-byte word per launch
    p->ws_queue = align_up(ws, 256);
    ws = p->ws_queue + 256;
  }
  p->ws_bytes = ws;

  int dev = -1, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FT_ERR_NO_DEVICE, "no HIP device");
  if (hipGetDevice(&dev) != hipSuccess) return fail(FT_ERR_NO_DEVICE, "no current HIP device");
  p->device = dev;
  char* scr = nullptr;   // the no-allocation peak call's scratch, resolved here once per device
  ft_status sst = scratch_for_device(dev, &scr);
  if (sst != FT_OK) return sst;

  if (!offsets.empty() && !p->chirpz && p->prec == FT_PREC_FP32) {
    // the queue schedule: every class's column length and row lengths need a queue kernel
    const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
    bool okq = (int)p->cls.size() * ns <= funnel::kQueueSegs;
    for (const auto& c : p->cls) {
      okq = okq && funnel::queue_col_kind(c.Np) >= 0;
      if (p->spaces & FT_SPACE_REGULAR) okq = okq && funnel::queue_row_kind(c.M) >= 0;
      if (p->spaces & FT_SPACE_INVERSE) okq = okq && funnel::queue_row_kind(c.N) >= 0;
    }
    if (okq) {
      const funnel::QueuePass kinds[3] = {funnel::QueuePass::R2C, funnel::QueuePass::C2R, funnel::QueuePass::ROW};
      for (int k = 0; k < 3 && okq; ++k)
        for (int sh = 0; sh < 2 && okq; ++sh)
          okq = funnel::queue_grid_size(kinds[k], sh, &p->qgrid[k][sh]) == hipSuccess && p->qgrid[k][sh] > 0;
    }
    p->queue_ok = okq;
  }

  std::vector<float2> host(ntw);
  for (auto& c : p->cls) {
    fill_twiddles(host.data() + c.tw_np, c.Np);
    fill_twiddles(host.data() + c.tw_m, c.M);
    fill_twiddles(host.data() + c.tw_n, c.N);
    if (p->prec != FT_PREC_FP32) {
      fill_mfma_lane_twiddles(host.data() + c.tw_np + c.Np, c.Np);
      fill_mfma_lane_twiddles(host.data() + c.tw_m + c.M, c.M);
      fill_mfma_lane_twiddles(host.data() + c.tw_n + c.N, c.N);
    }
    if (p->chirpz) {
      fill_twiddles(host.data() + c.tw_2m, 2 * c.M);
      fill_twiddles(host.data() + c.tw_2n, 2 * c.N);
    }
  }
  hipError_t e = hipMalloc(&p->tw, ntw * sizeof(float2));
  if (e != hipSuccess) return fail(FT_ERR_OUT_OF_MEMORY, "hipMalloc of twiddle tables: %s", hipGetErrorString(e));
  e = hipMemcpy(p->tw, host.data(), ntw * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy of twiddle tables");

  if (p->chirpz) {
    // per space and frequency row: the chirp spectrum (2W) and the chirp (W)
    size_t nch = 0;
    for (auto& c : p->cls) {
      if (p->spaces & FT_SPACE_REGULAR) {
        c.cz_m = nch;
        nch += (size_t)c.h * 2 * c.M;
        c.wz_m = nch;
        nch += (size_t)c.h * c.M;
      }
      if (p->spaces & FT_SPACE_INVERSE) {
        c.cz_n = nch;
        nch += (size_t)c.h * 2 * c.N;
        c.wz_n = nch;
        nch += (size_t)c.h * c.N;
      }
    }
    std::vector<float2> ch(nch);
    for (auto& c : p->cls) {
      if (p->spaces & FT_SPACE_REGULAR) funnel::chirp_tables(c.M, c.Np, c.h, ch.data() + c.cz_m, ch.data() + c.wz_m);
      if (p->spaces & FT_SPACE_INVERSE) funnel::chirp_tables(c.N, c.Np, c.h, ch.data() + c.cz_n, ch.data() + c.wz_n);
    }
    e = hipMalloc(&p->chirp, nch * sizeof(float2));
    if (e != hipSuccess) return fail(FT_ERR_OUT_OF_MEMORY, "hipMalloc of chirp tables: %s", hipGetErrorString(e));
    e = hipMemcpy(p->chirp, ch.data(), nch * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of chirp tables");
  }

  if (!offsets.empty()) {
    // one allocation: image offsets, plane offsets (int64) of all classes, then image indices (int32)
    size_t n = 0;
    for (auto& c : p->cls) n += c.count;
    std::vector<long long> l64(2 * n);
    std::vector<int> i32(n);
    size_t k = 0;
    for (size_t ci = 0; ci < p->cls.size(); ++ci)
      for (size_t j = 0; j < offsets[ci].size(); ++j, ++k) {
        l64[k] = offsets[ci][j].first;
        l64[n + k] = offsets[ci][j].second;
        i32[k] = p->cls[ci].images[j];
      }
    const size_t bytes = 2 * n * sizeof(long long) + n * sizeof(int);
    e = hipMalloc(&p->tables, bytes);
    if (e != hipSuccess) return fail(FT_ERR_OUT_OF_MEMORY, "hipMalloc of offset tables: %s", hipGetErrorString(e));
    char* t = static_cast<char*>(p->tables);
    e = hipMemcpy(t, l64.data(), 2 * n * sizeof(long long), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(t + 2 * n * sizeof(long long), i32.data(), n * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy of offset tables");
    size_t base = 0;
    for (auto& c : p->cls) {
      c.d_img_off = reinterpret_cast<const long long*>(t) + base;
      c.d_plane_off = reinterpret_cast<const long long*>(t) + n + base;
      c.d_gidx = reinterpret_cast<const int*>(t + 2 * n * sizeof(long long)) + base;
      base += c.count;
    }
  }
  if (p->cls.size() > 1) {
    if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
      return fail(FT_ERR_HIP, "hipEventCreate failed");
    for (auto& c : p->cls)
      if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess)
        return fail(FT_ERR_HIP, "stream or event creation failed");
  }
  return FT_OK;
}

}  // namespace

extern "C" {

const char* funnel_status_string(ft_status s) {
  switch (s) {
    case FT_OK: return "FT_OK";
    case FT_ERR_INVALID_ARG: return "FT_ERR_INVALID_ARG";
    case FT_ERR_UNSUPPORTED_SIZE: return "FT_ERR_UNSUPPORTED_SIZE";
    case FT_ERR_MISALIGNED: return "FT_ERR_MISALIGNED";
    case FT_ERR_WORKSPACE_TOO_SMALL: return "FT_ERR_WORKSPACE_TOO_SMALL";
    case FT_ERR_NO_DEVICE: return "FT_ERR_NO_DEVICE";
    case FT_ERR_HIP: return "FT_ERR_HIP";
    case FT_ERR_OUT_OF_MEMORY: return "FT_ERR_OUT_OF_MEMORY";
  }
  return "FT_ERR_UNKNOWN";
}

const char* funnel_last_error(void) { return g_err.c_str(); }

ft_status funnel_plan_create(const ft_plan_desc* d, ft_plan** out) {
  if (!d || !out) return fail(FT_ERR_INVALID_ARG, "desc and out must be non-NULL");
  *out = nullptr;
  if (d->batch < 1) return fail(FT_ERR_INVALID_ARG, "batch must be >= 1 (got %d)", d->batch);
  if (d->rows < 4 || d->cols < 4 || (d->rows & 1) || (d->cols & 1))
    return fail(FT_ERR_INVALID_ARG, "rows and cols must be even and >= 4 (got %d x %d)", d->rows, d->cols);
  if (d->spaces < FT_SPACE_REGULAR || d->spaces > FT_SPACE_BOTH)
    return fail(FT_ERR_INVALID_ARG, "spaces must be 1, 2 or 3 (got %d)", d->spaces);
  if (d->precision < FT_PREC_FP32 || d->precision > FT_PREC_FP16X3)
    return fail(FT_ERR_INVALID_ARG, "unknown precision %d", d->precision);
  if (d->flags & ~(uint32_t)FT_PLAN_NVMT_CHIRPZ) return fail(FT_ERR_INVALID_ARG, "unknown plan flags 0x%x", d->flags);
  const bool chirpz = (d->flags & FT_PLAN_NVMT_CHIRPZ) != 0;
  const long long N = d->rows, M = d->cols;
  const long long Np = d->padded_len == 0 ? N + M : d->padded_len;
  if (d->padded_len < 0 || (Np & 1) || Np < N + M)
    return fail(FT_ERR_INVALID_ARG, "padded_len must be 0 or even and >= rows+cols (got %d)", d->padded_len);
  ft_status st = validate_shape((int)N, (int)M, d->spaces, Np);
  if (st != FT_OK) return st;
  if (d->precision != FT_PREC_FP32) {
    // the matrix-core passes cover power-of-two lengths with a register-resident tile
    const char* what = nullptr;
    int len = 0;
    if (!funnel::col_variant_mask((int)Np, d->precision)) what = "padded length", len = (int)Np;
    else if ((d->spaces & FT_SPACE_REGULAR) && !funnel::row_variant_mask((int)M, d->precision))
      what = "row length (image width)", len = (int)M;
    else if ((d->spaces & FT_SPACE_INVERSE) && !funnel::row_variant_mask((int)N, d->precision))
      what = "row length (image height)", len = (int)N;
    if (what)
      return fail(FT_ERR_UNSUPPORTED_SIZE, "precision %d has no kernel for %s %d (powers of two only)", d->precision,
                  what, len);
  }

  if (chirpz) {
    if (d->precision != FT_PREC_FP32)
      return fail(FT_ERR_UNSUPPORTED_SIZE, "the chirp-z NVMT has FP32 kernels only (precision %d)", d->precision);
    if ((d->spaces & FT_SPACE_REGULAR) && !funnel::chirp_variant_mask((int)M))
      return fail(FT_ERR_UNSUPPORTED_SIZE, "no chirp-z kernel for row length (image width) %lld", M);
    if ((d->spaces & FT_SPACE_INVERSE) && !funnel::chirp_variant_mask((int)N))
      return fail(FT_ERR_UNSUPPORTED_SIZE, "no chirp-z kernel for row length (image height) %lld", N);
  }

  ft_plan* p = new (std::nothrow) ft_plan();
  if (!p) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->spaces = d->spaces;
  p->batch = d->batch;
  p->prec = d->precision;
  p->chirpz = chirpz;
  p->cls.resize(1);
  FtClass& c = p->cls[0];
  c.N = (int)N;
  c.M = (int)M;
  c.Np = (int)Np;
  c.count = d->batch;
  p->plane_elems = class_plane_floats(p->spaces, c);
  c.img_stride = N * M;
  c.plane_stride = (long long)p->plane_elems;
  p->image_extent = (size_t)d->batch * N * M;
  p->plane_extent = (size_t)d->batch * p->plane_elems;
  if ((long long)p->plane_extent > (1ll << 40)) {
    free_plan(p);
    return fail(FT_ERR_INVALID_ARG, "batch too large");
  }
  st = finish_plan(p, {});
  if (st != FT_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return ok();
}

ft_status funnel_plan_create_ragged(const ft_image_desc* images, int32_t count, int32_t spaces, ft_plan** out) {
  if (!images || !out) return fail(FT_ERR_INVALID_ARG, "images and out must be non-NULL");
  *out = nullptr;
  if (count < 1) return fail(FT_ERR_INVALID_ARG, "count must be >= 1 (got %d)", count);
  if (spaces < FT_SPACE_REGULAR || spaces > FT_SPACE_BOTH)
    return fail(FT_ERR_INVALID_ARG, "spaces must be 1, 2 or 3 (got %d)", spaces);
  std::map<std::pair<int, int>, int> index;
  std::vector<std::vector<std::pair<long long, long long>>> offs;
  ft_plan* p = new (std::nothrow) ft_plan();
  if (!p) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->spaces = spaces;
  p->batch = count;
  p->ragged = true;
  for (int i = 0; i < count; ++i) {
    const ft_image_desc& d = images[i];
    ft_status st = validate_shape(d.rows, d.cols, spaces, (long long)d.rows + d.cols);
    if (st == FT_OK && (d.image_offset < 0 || d.plane_offset < 0 || (d.image_offset & 3) || (d.plane_offset & 3)))
      st = fail(FT_ERR_MISALIGNED, "offsets must be non-negative multiples of 4 floats");
    if (st != FT_OK) {
      const std::string m = g_err;
      free_plan(p);
      return fail(st, "image %d: %s", i, m.c_str());
    }
    const auto key = std::make_pair(d.rows, d.cols);
    auto it = index.find(key);
    int ci;
    if (it == index.end()) {
      ci = (int)p->cls.size();
      index[key] = ci;
      p->cls.emplace_back();
      offs.emplace_back();
      FtClass& c = p->cls.back();
      c.N = d.rows;
      c.M = d.cols;
      c.Np = d.rows + d.cols;
    } else {
      ci = it->second;
    }
    FtClass& c = p->cls[ci];
    c.images.push_back(i);
    c.count += 1;
    offs[ci].emplace_back(d.image_offset, d.plane_offset);
    const size_t pf = class_plane_floats(spaces, c);
    p->image_extent = std::max(p->image_extent, (size_t)d.image_offset + (size_t)d.rows * d.cols);
    p->plane_extent = std::max(p->plane_extent, (size_t)d.plane_offset + pf);
  }
  p->plane_elems = p->plane_extent;
  ft_status st = finish_plan(p, offs);
  if (st != FT_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return ok();
}

void funnel_plan_destroy(ft_plan* p) { free_plan(p); }

ft_status funnel_workspace_size(const ft_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  *bytes = p->ws_bytes;
  return ok();
}

ft_status funnel_plane_elems(const ft_plan* p, size_t* n) {
  if (!p || !n) return fail(FT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  *n = p->plane_elems;
  return ok();
}

ft_status funnel_buffer_elems(const ft_plan* p, size_t* image_floats, size_t* plane_floats) {
  if (!p || !image_floats || !plane_floats) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  *image_floats = p->image_extent;
  *plane_floats = p->plane_extent;
  return ok();
}

ft_status funnel_padded_len(const ft_plan* p, int32_t* np) {
  if (!p || !np) return fail(FT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  if (p->ragged) return fail(FT_ERR_INVALID_ARG, "a ragged plan has one padded length per size class");
  *np = p->cls[0].Np;
  return ok();
}

ft_status funnel_forward(const ft_plan* p, const float* images, float* planes, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, images, planes, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  hipError_t e = enqueue_roles(p, kForwardOrder, images, planes, static_cast<char*>(ws),
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_adjoint(const ft_plan* p, const float* d_planes, float* d_images, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, d_planes, d_images, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  hipError_t e = enqueue_roles(p, kAdjointOrder, d_planes, d_images, static_cast<char*>(ws),
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

// ------------------------------------------------------------------ graphs

ft_status funnel_graph_create(const ft_plan* p, uint32_t what, const float* images, float* planes,
                              const float* d_planes, float* d_images, void* ws, size_t ws_bytes, ft_graph** out) {
  if (!p || !out) return fail(FT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  *out = nullptr;
  if (what == 0 || (what & ~(uint32_t)(FT_GRAPH_FORWARD | FT_GRAPH_ADJOINT)))
    return fail(FT_ERR_INVALID_ARG, "what must combine FT_GRAPH_FORWARD and FT_GRAPH_ADJOINT");
  ft_status st = FT_OK;
  if (what & FT_GRAPH_FORWARD) st = check_call(p, images, planes, ws, ws_bytes);
  if (st == FT_OK && (what & FT_GRAPH_ADJOINT)) st = check_call(p, d_planes, d_images, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  if (p->prof) return fail(FT_ERR_INVALID_ARG, "disable profiling before capturing a graph");
  ft_graph* g = new (std::nothrow) ft_graph();
  if (!g) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  g->device = p->device;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  hipError_t le = hipSuccess;
  if (e == hipSuccess) {
    if (what & FT_GRAPH_FORWARD) le = enqueue_roles(p, kForwardOrder, images, planes, static_cast<char*>(ws), cs);
    if (le == hipSuccess && (what & FT_GRAPH_ADJOINT))
      le = enqueue_roles(p, kAdjointOrder, d_planes, d_images, static_cast<char*>(ws), cs);
    e = hipStreamEndCapture(cs, &g->graph);
  }
  if (e == hipSuccess && le == hipSuccess) e = hipGraphInstantiateWithFlags(&g->exec, g->graph, 0);
  if (cs) (void)hipStreamDestroy(cs);
  if (e != hipSuccess || le != hipSuccess) {
    funnel_graph_destroy(g);
    return hip_fail(le != hipSuccess ? le : e, "graph capture");
  }
  *out = g;
  return ok();
}

ft_status funnel_graph_launch(const ft_graph* g, void* stream) {
  if (!g || !g->exec) return fail(FT_ERR_INVALID_ARG, "graph is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g->device)
    return fail(FT_ERR_NO_DEVICE, "graph was built on device %d", g->device);
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return ok();
}

void funnel_graph_destroy(ft_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ------------------------------------------------------------------ tuning

ft_status funnel_autotune(ft_plan* p, void* stream, ft_tune_result* out, int32_t cap, int32_t* n) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (cap < 0 || (cap > 0 && (!out || !n))) return fail(FT_ERR_INVALID_ARG, "bad result buffer");
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t big = std::max(p->image_extent, p->plane_extent) * sizeof(float);
  const size_t wsb = p->ws_bytes ? p->ws_bytes : 256;
  void *a = nullptr, *b = nullptr, *w = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (w) (void)hipFree(w);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&a, big) != hipSuccess || hipMalloc(&b, big) != hipSuccess || hipMalloc(&w, wsb) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_OUT_OF_MEMORY, "autotune scratch allocation failed");
  }
  if (hipMemsetAsync(a, 0, big, s) != hipSuccess || hipMemsetAsync(b, 0, big, s) != hipSuccess ||
      hipMemsetAsync(w, 0, wsb, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_HIP, "autotune set-up failed");
  }
  FtProfiler* saved = p->prof;
  p->prof = nullptr;
  int count = 0;
  // coordinate descent over the launches, two sweeps (a launch's best shape
  // can depend on its neighbours' shapes); results report the last sweep
  for (int sweep = 0; sweep < 2; ++sweep)
  for (size_t ci = 0; ci < p->cls.size(); ++ci) {
    FtClass& c = p->cls[ci];
    for (int r = 0; r < NROLES; ++r) {
      if (!role_active(p, r)) continue;
      const unsigned mask = role_mask(p, c, r);
      float best = 1e30f, first_ms = -1.f;
      int best_v = c.variant[r], tried = 0;
      for (int v = 0; v < funnel::kMaxVariants; ++v) {
        if (!(mask & (1u << v))) continue;
        // Score a variant by the time of the class's whole forward + adjoint
        // chain (the quantity a caller pays): a launch timed on its own, or
        // even inside the chain, misjudges how it overlaps with and warms the
        // caches for its neighbours.  Best of 7 chains after one warm-up.
        float ms_min = 1e30f;
        hipError_t e = hipSuccess;
        const int keep = c.variant[r];
        c.variant[r] = v;
        float* img = static_cast<float*>(a);
        float* pln = static_cast<float*>(b);
        for (int rep = 0; rep < 8 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, s);
          for (int k = 0; k < 12 && e == hipSuccess; ++k) {
            const int rr = k < 6 ? kForwardOrder[k] : kAdjointOrder[k - 6];
            if (!role_active(p, rr)) continue;
            const bool fwd = k < 6;
            e = run_role(p, c, rr, c.variant[rr], fwd ? img : pln, fwd ? pln : img, static_cast<char*>(w), s);
          }
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e == hipSuccess && rep > 0 && ms < ms_min) ms_min = ms;
        }
        c.variant[r] = keep;
        if (e != hipSuccess) {
          p->prof = saved;
          cleanup();
          return hip_fail(e, "autotune launch");
        }
        if (v == c.variant[r]) first_ms = ms_min;
        ++tried;
        if (ms_min < best) {
          best = ms_min;
          best_v = v;
        }
      }
      c.variant[r] = best_v;
      if (sweep == 0) continue;
      if (count < cap) {
        std::memset(&out[count], 0, sizeof(ft_tune_result));
        std::snprintf(out[count].name, sizeof(out[count].name), "%s", role_label(p, (int)ci, r).c_str());
        out[count].variant = best_v;
        out[count].n_tried = tried;
        out[count].ms = best;
        out[count].ms_default = first_ms;
      }
      ++count;
    }
  }
  if (p->ragged && p->queue_ok) {
    // the schedule: the classes' tuned launches on their streams, or the
    // queue's persistent launches (each column launch's tile shape tried)
    auto chain_ms = [&](float* best_ms) -> hipError_t {
      float m = 1e30f;
      hipError_t e = hipSuccess;
      float* img = static_cast<float*>(a);
      float* pln = static_cast<float*>(b);
      for (int rep = 0; rep < 8 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = enqueue_roles(p, kForwardOrder, img, pln, static_cast<char*>(w), s);
        if (e == hipSuccess) e = enqueue_roles(p, kAdjointOrder, pln, img, static_cast<char*>(w), s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && ms < m) m = ms;
      }
      *best_ms = m;
      return e;
    };
    float t_streams = 0.f, t_queue = 0.f, t = 0.f;
    p->schedule = FT_SCHEDULE_CLASS_STREAMS;
    hipError_t e = chain_ms(&t_streams);
    p->schedule = FT_SCHEDULE_QUEUE;
    for (int ql = 0; ql < kQueueLaunches; ++ql) p->qshape[ql] = 0;
    if (e == hipSuccess) e = chain_ms(&t_queue);
    int tried = 2;
    for (int ql : {QF_A, QF_C, QA_CT, QA_AT_INV, QA_AT_REG}) {
      if (e != hipSuccess) break;
      p->qshape[ql] = 1;
      e = chain_ms(&t);
      ++tried;
      if (e == hipSuccess && t < t_queue) t_queue = t;
      else p->qshape[ql] = 0;
    }
    if (e != hipSuccess) {
      p->schedule = FT_SCHEDULE_CLASS_STREAMS;
      p->prof = saved;
      cleanup();
      return hip_fail(e, "autotune launch");
    }
    p->schedule = t_queue < t_streams ? FT_SCHEDULE_QUEUE : FT_SCHEDULE_CLASS_STREAMS;
    if (count < cap) {
      std::memset(&out[count], 0, sizeof(ft_tune_result));
      std::snprintf(out[count].name, sizeof(out[count].name), "schedule");
      out[count].variant = p->schedule;
      out[count].n_tried = tried;
      out[count].ms = p->schedule == FT_SCHEDULE_QUEUE ? t_queue : t_streams;
      out[count].ms_default = t_streams;
    }
    ++count;
  }
  p->prof = saved;
  cleanup();
  if (n) *n = count < cap ? count : cap;
  return ok();
}

ft_status funnel_plan_variants(const ft_plan* p, int32_t* variants, int32_t cap) {
  if (!p || !variants || cap < 1) return fail(FT_ERR_INVALID_ARG, "plan and variants must be non-NULL");
  int k = 0;
  for (const auto& c : p->cls)
    for (int r = 0; r < NROLES && k < cap; ++r, ++k) variants[k] = role_active(p, r) ? c.variant[r] : -1;
  return ok();
}

ft_status funnel_plan_set_variant(ft_plan* p, int32_t role, int32_t variant) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (role < 0 || role >= (int)p->cls.size() * NROLES)
    return fail(FT_ERR_INVALID_ARG, "role must be in 0..%d", (int)p->cls.size() * NROLES - 1);
  const int ci = role / NROLES, r = role % NROLES;
  if (variant < 0 || variant >= funnel::kMaxVariants || !(role_mask(p, p->cls[ci], r) & (1u << variant)))
    return fail(FT_ERR_INVALID_ARG, "variant %d has no kernel for role %s", variant, kRoleName[r]);
  p->cls[ci].variant[r] = variant;
  return ok();
}

ft_status funnel_plan_set_schedule(ft_plan* p, int32_t schedule) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (schedule != FT_SCHEDULE_CLASS_STREAMS && schedule != FT_SCHEDULE_QUEUE)
    return fail(FT_ERR_INVALID_ARG, "unknown schedule %d", schedule);
  if (schedule == FT_SCHEDULE_QUEUE && !p->ragged)
    return fail(FT_ERR_INVALID_ARG, "the queue schedule is for ragged plans");
  if (schedule == FT_SCHEDULE_QUEUE && !p->queue_ok)
    return fail(FT_ERR_UNSUPPORTED_SIZE, "a length of this plan has no queue kernel");
  p->schedule = schedule;
  return ok();
}

ft_status funnel_plan_schedule(const ft_plan* p, int32_t* schedule) {
  if (!p || !schedule) return fail(FT_ERR_INVALID_ARG, "plan and schedule must be non-NULL");
  *schedule = p->schedule;
  return ok();
}

ft_status funnel_plan_classes(const ft_plan* p, int32_t* n) {
  if (!p || !n) return fail(FT_ERR_INVALID_ARG, "plan and n must be non-NULL");
  *n = (int32_t)p->cls.size();
  return ok();
}

// ------------------------------------------------------------------ timing

}  // extern "C"

namespace {

ft_status profiler_enable(FtProfiler*& slot, int32_t max_records) {
  if (max_records < 1 || max_records > (1 << 20))
    return fail(FT_ERR_INVALID_ARG, "max_records must be in 1..2^20 (got %d)", max_records);
  FtProfiler* pr = new (std::nothrow) FtProfiler();
  if (!pr) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  pr->cap = max_records;
  pr->ev0.resize(max_records);
  pr->ev1.resize(max_records);
  pr->name.assign(max_records, std::string());
  pr->bytes.assign(max_records, 0.0);
  for (int i = 0; i < max_records; ++i) {
    if (hipEventCreate(&pr->ev0[i]) != hipSuccess || hipEventCreate(&pr->ev1[i]) != hipSuccess) {
      pr->ev0.resize(i);
      pr->ev1.resize(i);
      free_profiler(pr);
      return fail(FT_ERR_HIP, "hipEventCreate failed");
    }
  }
  free_profiler(slot);
  slot = pr;
  return ok();
}

ft_status profiler_read(FtProfiler* pr, ft_kernel_time* out, int32_t cap, int32_t* n) {
  if (!out || !n || cap < 1) return fail(FT_ERR_INVALID_ARG, "out and n must be non-NULL, cap >= 1");
  *n = 0;
  if (!pr) return fail(FT_ERR_INVALID_ARG, "profiling is not enabled on this plan");
  int cnt = 0;
  for (int i = 0; i < pr->used; ++i) {
    hipError_t e = hipEventSynchronize(pr->ev1[i]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, pr->ev0[i], pr->ev1[i]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    int k = 0;
    while (k < cnt && pr->name[i] != out[k].name) ++k;
    if (k == cnt) {
      if (cnt == cap) continue;
      std::memset(&out[k], 0, sizeof(ft_kernel_time));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", pr->name[i].c_str());
      out[k].bytes_per_launch = pr->bytes[i];
      ++cnt;
    }
    out[k].launches += 1;
    out[k].total_ms += ms;
  }
  pr->used = 0;
  *n = cnt;
  return ok();
}

}  // namespace

extern "C" {

ft_status funnel_profile_enable(ft_plan* p, int32_t max_records) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  return profiler_enable(p->prof, max_records);
}

ft_status funnel_profile_read(ft_plan* p, ft_kernel_time* out, int32_t cap, int32_t* n) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  return profiler_read(p->prof, out, cap, n);
}

ft_status funnel_profile_disable(ft_plan* p) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  free_profiler(p->prof);
  p->prof = nullptr;
  return ok();
}

// ------------------------------------------------------------------ peaks

ft_status funnel_peaks_workspace_size(const ft_plan* p, int32_t K, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  size_t total = 0;
  for (const auto& c : p->cls) {
    int tiles = 0;
    if (p->spaces & FT_SPACE_REGULAR) tiles = funnel::peaks_tiles(c.Np, c.M);
    if (p->spaces & FT_SPACE_INVERSE) tiles = std::max(tiles, funnel::peaks_tiles(c.Np, c.N));
    total += align_up(funnel::peaks_workspace_bytes(c.count * ns, tiles, K), 256);
  }
  *bytes = total;
  return ok();
}

}  // extern "C"

namespace {

// Host-side checks of a peak call, everything but the workspace.
ft_status peaks_args(const ft_plan* p, const float* planes, int32_t K, float threshold, int32_t radius,
                     uint32_t flags, const ft_peak* peaks, const int32_t* n_found) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!planes || !peaks || !n_found) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (radius < 1 || radius > 8) return fail(FT_ERR_INVALID_ARG, "radius must be in 1..8 (got %d)", radius);
  if (std::isnan(threshold)) return fail(FT_ERR_INVALID_ARG, "threshold is NaN");
  if (flags & ~(uint32_t)(FT_PEAK_CLAMP_BORDER | FT_PEAK_KEEP_PAD_BOUNDARY))
    return fail(FT_ERR_INVALID_ARG, "unknown peak flags 0x%x", flags);
  if (!aligned16(planes) || !aligned16(peaks) || !aligned16(n_found))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  return FT_OK;
}

// Enqueue the peak kernels of every size class; class c's partial lists and
// cutoffs take the next peaks_workspace_bytes of w.
hipError_t peaks_enqueue(const ft_plan* p, const float* planes, int32_t K, float threshold, int32_t radius,
                         uint32_t flags, ft_peak* peaks, int32_t* n_found, char* w, hipStream_t s) {
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  const bool fork = p->cls.size() > 1;
  hipError_t e = hipSuccess;
  if (fork) e = hipEventRecord(p->fork, s);
  for (size_t ci = 0; ci < p->cls.size() && e == hipSuccess; ++ci) {
    const FtClass& c = p->cls[ci];
    hipStream_t cs = fork ? c.stream : s;
    if (fork) e = hipStreamWaitEvent(cs, p->fork, 0);
    int rows[2], cols[2], himg[2], tiles = 0, k = 0;
    long long off[2];
    if (p->spaces & FT_SPACE_REGULAR) {
      rows[k] = c.Np; cols[k] = c.M; himg[k] = c.N; off[k] = 0; ++k;
      tiles = funnel::peaks_tiles(c.Np, c.M);
    }
    if (p->spaces & FT_SPACE_INVERSE) {
      rows[k] = c.Np; cols[k] = c.N; himg[k] = c.M; off[k] = (long long)c.off_inv_plane; ++k;
      tiles = std::max(tiles, funnel::peaks_tiles(c.Np, c.N));
    }
    const funnel::ImgMap map{0, c.plane_stride, nullptr, c.d_plane_off};
    if (e == hipSuccess)
      e = funnel::launch_peaks(planes, map, c.d_gidx, c.count, ns, (p->spaces & FT_SPACE_REGULAR) ? 0 : 1, rows, cols,
                               himg, off, K, threshold, radius,
                               (flags & FT_PEAK_CLAMP_BORDER) ? 0 : 1, (flags & FT_PEAK_KEEP_PAD_BOUNDARY) ? 1 : 0,
                               peaks, n_found, w, cs);
    w += align_up(funnel::peaks_workspace_bytes(c.count * ns, tiles, K), 256);
    if (fork && e == hipSuccess) e = hipEventRecord(c.done, cs);
  }
  for (size_t ci = 0; fork && ci < p->cls.size() && e == hipSuccess; ++ci)
    e = hipStreamWaitEvent(s, p->cls[ci].done, 0);
  return e;
}

}  // namespace

extern "C" {

ft_status funnel_peaks(const ft_plan* p, const float* planes, int32_t K, float threshold, int32_t radius,
                       uint32_t flags, ft_peak* peaks, int32_t* n_found, void* ws, size_t ws_bytes, void* stream) {
  ft_status st = peaks_args(p, planes, K, threshold, radius, flags, peaks, n_found);
  if (st != FT_OK) return st;
  if (!ws) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  if (!aligned16(ws)) return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  size_t need = 0;
  if ((st = funnel_peaks_workspace_size(p, K, &need)) != FT_OK) return st;
  if (ws_bytes < need) return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  hipError_t e = peaks_enqueue(p, planes, K, threshold, radius, flags, peaks, n_found, static_cast<char*>(ws),
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_peaks_noalloc(const ft_plan* p, const float* planes, int32_t K, float threshold, int32_t radius,
                               uint32_t flags, ft_peak* peaks, int32_t* n_found, void* stream) {
  ft_status st = peaks_args(p, planes, K, threshold, radius, flags, peaks, n_found);
  if (st != FT_OK) return st;
  size_t need = 0;
  if ((st = funnel_peaks_workspace_size(p, K, &need)) != FT_OK) return st;
  if (need > kPeakScratchBytes)
    return fail(FT_ERR_WORKSPACE_TOO_SMALL,
                "this plan and K need %zu bytes of peak scratch, the static scratch holds %zu; "
                "use funnel_peaks with a workspace", need, kPeakScratchBytes);
  if ((st = check_device(p)) != FT_OK) return st;
  char* w = nullptr;
  if ((st = scratch_for_device(p->device, &w)) != FT_OK) return st;
  (void)hipGetLastError();
  hipError_t e = peaks_enqueue(p, planes, K, threshold, radius, flags, peaks, n_found, w,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_verify(const ft_plan* p, const float* images, const ft_peak* peaks, const int32_t* n_found,
                        int32_t K, int32_t half_width, float min_contrast, int32_t min_length, ft_line_check* out,
                        void* stream) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!images || !peaks || !n_found || !out) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (half_width < 1 || half_width > 3) return fail(FT_ERR_INVALID_ARG, "half_width must be in 1..3 (got %d)", half_width);
  if (std::isnan(min_contrast)) return fail(FT_ERR_INVALID_ARG, "min_contrast is NaN");
  if (min_length < 0) return fail(FT_ERR_INVALID_ARG, "min_length must be >= 0 (got %d)", min_length);
  if (!aligned16(images) || !aligned16(peaks) || !aligned16(n_found) || !aligned16(out))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  hipError_t e = hipSuccess;
  for (size_t ci = 0; ci < p->cls.size() && e == hipSuccess; ++ci) {
    const FtClass& c = p->cls[ci];
    const funnel::ImgMap map{c.img_stride, 0, c.d_img_off, nullptr};
    e = funnel::launch_verify(images, map, c.d_gidx, c.count, ns, c.N, c.M, peaks, n_found, K, half_width,
                              min_contrast, min_length, out, s);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

namespace {
// refinement workspace: the transform's spectra, the row sums A (3 complex
// per row, peak and space), the iteration state
struct RefineLayout {
  size_t a_off, st_off, total;
};
RefineLayout refine_layout(const ft_plan* p, int K) {
  const FtClass& c = p->cls[0];
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  RefineLayout L;
  L.a_off = align_up(p->ws_bytes, 256);
  L.st_off = align_up(L.a_off + (size_t)c.count * ns * K * 3 * (size_t)c.h * sizeof(float2), 256);
  L.total = align_up(L.st_off + (size_t)c.count * ns * K * funnel::refine_state_bytes(), 256);
  return L;
}
}  // namespace

ft_status funnel_refine_workspace_size(const ft_plan* p, int32_t K, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (p->cls.size() != 1 || p->ragged) return fail(FT_ERR_INVALID_ARG, "refinement needs a uniform plan");
  *bytes = refine_layout(p, K).total;
  return ok();
}

ft_status funnel_refine(const ft_plan* p, const float* images, const ft_peak* peaks, const int32_t* n_found,
                        int32_t K, int32_t iters, ft_refined* out, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!images || !peaks || !n_found || !out || !ws) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (iters < 0 || iters > 16) return fail(FT_ERR_INVALID_ARG, "iters must be in 0..16 (got %d)", iters);
  if (p->cls.size() != 1 || p->ragged) return fail(FT_ERR_INVALID_ARG, "refinement needs a uniform plan");
  const FtClass& c = p->cls[0];
  if (((p->spaces & FT_SPACE_REGULAR) && !funnel::refine_length_supported(c.M)) ||
      ((p->spaces & FT_SPACE_INVERSE) && !funnel::refine_length_supported(c.N)))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "refinement needs power-of-two row lengths in 64..4096 (%d x %d)", c.N, c.M);
  if (!aligned16(images) || !aligned16(peaks) || !aligned16(n_found) || !aligned16(out) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  const RefineLayout L = refine_layout(p, K);
  if (ws_bytes < L.total) return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  const int B = c.count, h = c.h;
  float2* Abuf = reinterpret_cast<float2*>(w + L.a_off);
  void* state = w + L.st_off;
  hipError_t e = hipSuccess;
  // the resampled rows g of each space: pass A of the forward, then the
  // interpolation of pass B alone (linear NVMT), or pass B and the inverse x'
  // DFT (chirp-z NVMT, whose resampling is band-limited)
  struct Sp { int role_a, role_b, W, space_id; size_t off; size_t tw; };
  Sp sp[2];
  int k = 0;
  if (p->spaces & FT_SPACE_REGULAR) sp[k++] = {FA_REG, FB_REG, c.M, 0, c.ws_reg, c.tw_m};
  if (p->spaces & FT_SPACE_INVERSE) sp[k++] = {FA_INV, FB_INV, c.N, 1, c.ws_inv, c.tw_n};
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    e = run_role(p, c, sp[i].role_a, c.variant[sp[i].role_a], images, nullptr, w, s);
    float2* rows = reinterpret_cast<float2*>(w + sp[i].off);
    if (!p->chirpz) {
      if (e == hipSuccess) e = funnel::launch_row_lerp(sp[i].W, rows, h, c.Np, (long long)h * sp[i].W, B, s);
    } else {
      if (e == hipSuccess) e = run_role(p, c, sp[i].role_b, c.variant[sp[i].role_b], nullptr, nullptr, w, s);
      if (e == hipSuccess)
        e = funnel::launch_row_idft(sp[i].W, rows, h, (long long)h * sp[i].W, p->tw + sp[i].tw, B, s);
    }
  }
  if (e == hipSuccess)
    e = funnel::launch_refine_init(peaks, n_found, B, ns, K, sp[0].W, ns > 1 ? sp[1].W : sp[0].W, c.Np, state, s);
  for (int it = 0; it <= iters && e == hipSuccess; ++it)
    for (int i = 0; i < ns && e == hipSuccess; ++i)
      e = funnel::launch_refine_iter(reinterpret_cast<const float2*>(w + sp[i].off), (long long)h * sp[i].W, h,
                                     sp[i].W, i, ns, K, B, n_found, state, Abuf, c.Np, sp[i].space_id, c.N, c.M,
                                     it == iters ? 1 : 0, out, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ volumes (App. A)
//
// Per parameter space four launches: A (DFT along the space's depth axis of
// its R*C lines, the image pass A; columns of the volume for the z space,
// its rows for the x space, the rows of the slice-transposed volume for the
// y space), Bx (NVMT along the columns + DFT along x', the image row pass
// with R rows per ratio), By (NVMT along the rows + DFT along y',
// funnel_volume.hip) and C (Hermitian inverse DFT along omega_3, the image
// pass C), all in place on one half spectrum of h * R * C complex values per
// volume, which the spaces use one after the other.

enum VRole { VA, VBX, VBY, VC, NVROLES };
constexpr int kVSpaces = 3;   // z, x, y
static const char* const kVRoleName[kVSpaces][NVROLES] = {
    {"volume.A", "volume.Bx", "volume.By", "volume.C"},
    {"volume.x.A", "volume.x.Bx", "volume.x.By", "volume.x.C"},
    {"volume.y.A", "volume.y.Bx", "volume.y.By", "volume.y.C"}};

struct VSpace {
  bool on = false;
  int D = 0, R = 0, C = 0;      // depth, rows and columns of the space
  long long param_off = 0;      // floats from a volume's parameter block to this space's
  long long spec_elems = 0;     // h * R * C complex values per volume
  size_t tw_r = 0, tw_c = 0;    // twiddles of the y' (length R) and x' (length C) passes
  int variant[NVROLES] = {};
};

struct ft_volume_plan {
  FtProfiler* prof = nullptr;
  int device = 0;
  int batch = 0, Nz = 0, Ny = 0, Nx = 0, Lp = 0, h = 0;
  float2* tw = nullptr;         // twiddles of lengths Lp, Nx, Ny, Nz
  size_t tw_l = 0;
  long long vol_elems = 0, param_elems = 0;   // per volume; param_elems over all spaces
  size_t ws_tp_off = 0;         // byte offset of the slice-transposed volumes (y space)
  size_t ws_bytes = 0;
  VSpace sp[kVSpaces];
};

namespace {

unsigned vrole_mask(const ft_volume_plan* p, int si, int r) {
  const VSpace& q = p->sp[si];
  if (!q.on) return 0;
  switch (r) {
    case VA: case VC: return funnel::col_variant_mask(p->Lp, FT_PREC_FP32);
    case VBX: return funnel::row_variant_mask(q.C, FT_PREC_FP32);
    case VBY: return funnel::ycol_variant_mask(q.R);
  }
  return 0;
}

// algorithmic HBM bytes of one launch (each input read once, each output written once)
double vrole_bytes(const ft_volume_plan* p, int si, int r) {
  const VSpace& q = p->sp[si];
  const double B = p->batch, lines = (double)q.R * q.C, h = p->h;
  switch (r) {
    case VA: return B * (4.0 * q.D * lines + 8.0 * h * lines);
    case VBX: case VBY: return B * 16.0 * h * lines;
    case VC: return B * (8.0 * h * lines + 4.0 * p->Lp * lines);
  }
  return 0.0;
}

hipError_t run_vrole(const ft_volume_plan* p, int si, int r, int v, const float* src, float* dst, char* w,
                     hipStream_t s) {
  const VSpace& q = p->sp[si];
  float2* S = reinterpret_cast<float2*>(w);
  const int lines = q.R * q.C;
  const long long ss = q.spec_elems;
  using funnel::ImgMap;
  switch (r) {
    case VA: {
      // z: the volume's columns; x: its rows; y: the rows of its slice-transposed copy
      const float* in = si == 2 ? reinterpret_cast<const float*>(w + p->ws_tp_off) : src;
      return funnel::launch_r2c(p->Lp, v, FT_PREC_FP32, si != 0, in, S, lines, q.D, (p->Lp - q.D) / 2,
                                ImgMap{p->vol_elems, ss, nullptr, nullptr}, 1.0f, p->tw + p->tw_l, p->batch, s);
    }
    case VBX:
      return funnel::launch_row(q.C, v, FT_PREC_FP32, false, S, p->Lp, p->h, q.R, ss, p->tw + q.tw_c, p->batch, s);
    case VBY: return funnel::launch_ycol(q.R, v, S, p->Lp, p->h, q.C, ss, p->tw + q.tw_r, p->batch, s);
    case VC:
      return funnel::launch_c2r(p->Lp, v, FT_PREC_FP32, false, false, S, dst + q.param_off, lines, 0, p->Lp,
                                ImgMap{ss, p->param_elems, nullptr, nullptr}, 1.0f / p->Lp, p->tw + p->tw_l,
                                p->batch, s);
  }
  return hipErrorInvalidValue;
}

hipError_t enqueue_volume(const ft_volume_plan* p, const float* src, float* dst, char* w, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int si = 0; si < kVSpaces && e == hipSuccess; ++si) {
    if (!p->sp[si].on) continue;
    if (si == 2)
      e = timed(p, s, "volume.y.T", 8.0 * p->batch * p->vol_elems, [&] {
        return funnel::launch_transpose_slices(src, reinterpret_cast<float*>(w + p->ws_tp_off), p->batch * p->Nz,
                                               p->Ny, p->Nx, s);
      });
    for (int r = 0; r < NVROLES && e == hipSuccess; ++r)
      e = timed(p, s, kVRoleName[si][r], vrole_bytes(p, si, r),
                [&] { return run_vrole(p, si, r, p->sp[si].variant[r], src, dst, w, s); });
  }
  return e;
}

ft_status check_volume_device(const ft_volume_plan* p) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FT_ERR_NO_DEVICE, "no HIP device");
  if (dev != p->device) return fail(FT_ERR_NO_DEVICE, "plan was created on device %d, current is %d", p->device, dev);
  return FT_OK;
}

void free_volume_plan(ft_volume_plan* p) {
  if (!p) return;
  free_profiler(p->prof);
  if (p->tw) (void)hipFree(p->tw);
  delete p;
}

int n_vspaces(const ft_volume_plan* p) {
  int n = 0;
  for (const auto& q : p->sp) n += q.on ? 1 : 0;
  return n;
}

}  // namespace

extern "C" {

ft_status funnel_volume_plan_create(const ft_volume_desc* d, ft_volume_plan** out) {
  if (!d || !out) return fail(FT_ERR_INVALID_ARG, "desc and out must be non-NULL");
  *out = nullptr;
  if (d->batch < 1) return fail(FT_ERR_INVALID_ARG, "batch must be >= 1 (got %d)", d->batch);
  if (d->depth < 4 || d->rows < 4 || d->cols < 4 || (d->depth & 1) || (d->rows & 1) || (d->cols & 1))
    return fail(FT_ERR_INVALID_ARG, "depth, rows and cols must be even and >= 4 (got %d x %d x %d)", d->depth,
                d->rows, d->cols);
  if (d->spaces < 1 || d->spaces > FT_VOL_SPACE_ALL)
    return fail(FT_ERR_INVALID_ARG, "spaces must be a non-empty set of FT_VOL_SPACE_Z/X/Y (got %d)", d->spaces);
  if (d->flags != 0) return fail(FT_ERR_INVALID_ARG, "unknown volume plan flags 0x%x", d->flags);
  const long long Nz = d->depth, Ny = d->rows, Nx = d->cols;
  const long long Lp = d->padded_len == 0 ? Nz + Ny + Nx : d->padded_len;
  if (d->padded_len < 0 || (Lp & 1) || Lp < Nz + Ny + Nx)
    return fail(FT_ERR_INVALID_ARG, "padded_len must be 0 or even and >= depth+rows+cols (got %d)", d->padded_len);
  if (Lp > (1 << 20) || Nx > (1 << 20) || Ny > (1 << 20) || Nz > (1 << 20))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "transform length too large");
  if (!funnel::length_supported((int)Lp) || !funnel::col_variant_mask((int)Lp, FT_PREC_FP32))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for padded depth %lld", Lp);
  // (depth, rows, cols) of the z, x and y spaces
  const long long geo[kVSpaces][3] = {{Nz, Ny, Nx}, {Nx, Nz, Ny}, {Ny, Nz, Nx}};
  static const char* const sname[kVSpaces] = {"z", "x", "y"};
  for (int si = 0; si < kVSpaces; ++si) {
    if (!(d->spaces & (1 << si))) continue;
    const long long R = geo[si][1], C = geo[si][2];
    if (!funnel::length_supported((int)C) || !funnel::row_variant_mask((int)C, FT_PREC_FP32))
      return fail(FT_ERR_UNSUPPORTED_SIZE, "%s space: no x' pass kernel for row length %lld", sname[si], C);
    if (!funnel::ycol_variant_mask((int)R))
      return fail(FT_ERR_UNSUPPORTED_SIZE, "%s space: no y' pass kernel for column length %lld", sname[si], R);
    // the kernels address one volume's parameter block and half spectrum of
    // a space with 32-bit byte offsets
    if (Lp * R * C * 4 >= (1ll << 31))
      return fail(FT_ERR_UNSUPPORTED_SIZE, "%s space: per-volume parameter volumes of %lld x %lld x %lld exceed 2 GiB",
                  sname[si], Lp, R, C);
  }

  ft_volume_plan* p = new (std::nothrow) ft_volume_plan();
  if (!p) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->batch = d->batch;
  p->Nz = (int)Nz;
  p->Ny = (int)Ny;
  p->Nx = (int)Nx;
  p->Lp = (int)Lp;
  p->h = (int)Lp / 2 - 1;
  p->vol_elems = Nz * Ny * Nx;
  // twiddles: Lp, then Nx, Ny, Nz
  p->tw_l = 0;
  const size_t tw_x = (size_t)Lp, tw_y = tw_x + (size_t)Nx, tw_z = tw_y + (size_t)Ny, ntw = tw_z + (size_t)Nz;
  const size_t tw_of[kVSpaces][2] = {{tw_y, tw_x}, {tw_z, tw_y}, {tw_z, tw_x}};   // (rows, cols) per space
  size_t spec = 0;
  long long off = 0;
  for (int si = 0; si < kVSpaces; ++si) {
    VSpace& q = p->sp[si];
    q.on = (d->spaces & (1 << si)) != 0;
    if (!q.on) continue;
    q.D = (int)geo[si][0];
    q.R = (int)geo[si][1];
    q.C = (int)geo[si][2];
    q.param_off = off;
    off += Lp * q.R * q.C;
    q.spec_elems = (long long)p->h * q.R * q.C;
    q.tw_r = tw_of[si][0];
    q.tw_c = tw_of[si][1];
    const size_t b = (size_t)p->batch * q.spec_elems * sizeof(float2);
    spec = b > spec ? b : spec;
    for (int r = 0; r < NVROLES; ++r) {
      const unsigned m = vrole_mask(p, si, r);
      for (int v = 0; v < funnel::kMaxVariants; ++v)
        if (m & (1u << v)) {
          q.variant[r] = v;
          break;
        }
    }
    // the y' pass: prefer a tile whose column count divides the width
    for (int v = 0; v < funnel::kMaxVariants; ++v)
      if ((vrole_mask(p, si, VBY) & (1u << v)) && q.C % funnel::ycol_lines(v) == 0) {
        q.variant[VBY] = v;
        break;
      }
  }
  p->param_elems = off;
  p->ws_tp_off = align_up(spec, 256);
  p->ws_bytes = p->ws_tp_off + (p->sp[2].on ? align_up((size_t)p->batch * p->vol_elems * sizeof(float), 256) : 0);

  int dev = -1, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    free_volume_plan(p);
    return fail(FT_ERR_NO_DEVICE, "no HIP device");
  }
  if (hipGetDevice(&dev) != hipSuccess) {
    free_volume_plan(p);
    return fail(FT_ERR_NO_DEVICE, "no current HIP device");
  }
  p->device = dev;
  std::vector<float2> host(ntw);
  fill_twiddles(host.data(), (int)Lp);
  fill_twiddles(host.data() + tw_x, (int)Nx);
  fill_twiddles(host.data() + tw_y, (int)Ny);
  fill_twiddles(host.data() + tw_z, (int)Nz);
  hipError_t e = hipMalloc(&p->tw, ntw * sizeof(float2));
  if (e != hipSuccess) {
    p->tw = nullptr;
    free_volume_plan(p);
    return fail(FT_ERR_OUT_OF_MEMORY, "hipMalloc of twiddle tables: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(p->tw, host.data(), ntw * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_volume_plan(p);
    return hip_fail(e, "hipMemcpy of twiddle tables");
  }
  *out = p;
  return ok();
}

void funnel_volume_plan_destroy(ft_volume_plan* p) { free_volume_plan(p); }

ft_status funnel_volume_padded_len(const ft_volume_plan* p, int32_t* nzp) {
  if (!p || !nzp) return fail(FT_ERR_INVALID_ARG, "plan and nzp must be non-NULL");
  *nzp = p->Lp;
  return ok();
}

ft_status funnel_volume_param_elems(const ft_volume_plan* p, size_t* floats_per_volume) {
  if (!p || !floats_per_volume) return fail(FT_ERR_INVALID_ARG, "plan and floats_per_volume must be non-NULL");
  *floats_per_volume = (size_t)p->param_elems;
  return ok();
}

ft_status funnel_volume_workspace_size(const ft_volume_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  *bytes = p->ws_bytes;
  return ok();
}

ft_status funnel_volume_forward(const ft_volume_plan* p, const float* volumes, float* params, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!volumes || !params || !ws) return fail(FT_ERR_INVALID_ARG, "volumes, params and workspace must be non-NULL");
  if (!aligned16(volumes) || !aligned16(params) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  if (ws_bytes < p->ws_bytes)
    return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, p->ws_bytes);
  ft_status st = check_volume_device(p);
  if (st != FT_OK) return st;
  const hipError_t e = enqueue_volume(p, volumes, params, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_volume_peaks_workspace_size(const ft_volume_plan* p, int32_t K, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  size_t need = 0;
  for (const auto& q : p->sp) {
    if (!q.on) continue;
    const size_t b = funnel::vpeaks_workspace_bytes(p->batch, funnel::vpeaks_tiles(p->Lp, q.R, q.C), K);
    need = b > need ? b : need;
  }
  *bytes = need;
  return ok();
}

ft_status funnel_volume_peaks(const ft_volume_plan* p, const float* params, int32_t K, float threshold, int32_t radius,
                              uint32_t flags, ft_plane_peak* peaks, int32_t* n_found, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!params || !peaks || !n_found || !ws)
    return fail(FT_ERR_INVALID_ARG, "params, peaks, n_found and workspace must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (radius < 1 || radius > 2) return fail(FT_ERR_INVALID_ARG, "radius must be 1 or 2 (got %d)", radius);
  if (std::isnan(threshold)) return fail(FT_ERR_INVALID_ARG, "threshold is NaN");
  if (flags & ~(uint32_t)(FT_PEAK_CLAMP_BORDER | FT_PEAK_KEEP_PAD_BOUNDARY))
    return fail(FT_ERR_INVALID_ARG, "unknown peak flags 0x%x", flags);
  if (!aligned16(params) || !aligned16(peaks) || !aligned16(n_found) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  size_t need = 0;
  ft_status st = funnel_volume_peaks_workspace_size(p, K, &need);
  if (st != FT_OK) return st;
  if (ws_bytes < need) return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  st = check_volume_device(p);
  if (st != FT_OK) return st;
  const int ns = n_vspaces(p);
  hipError_t e = hipSuccess;
  for (int si = 0, k = 0; si < kVSpaces && e == hipSuccess; ++si) {
    const VSpace& q = p->sp[si];
    if (!q.on) continue;
    e = funnel::launch_vpeaks(params + q.param_off, p->param_elems, p->batch, p->Lp, q.R, q.C, q.D, K, threshold,
                              radius, (flags & FT_PEAK_CLAMP_BORDER) ? 0 : 1,
                              (flags & FT_PEAK_KEEP_PAD_BOUNDARY) ? 1 : 0, ns, k++, si, peaks, n_found, ws,
                              static_cast<hipStream_t>(stream));
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_volume_variants(const ft_volume_plan* p, int32_t* variants, int32_t cap) {
  if (!p || !variants || cap < 1) return fail(FT_ERR_INVALID_ARG, "plan and variants must be non-NULL, cap >= 1");
  for (int k = 0; k < kVSpaces * NVROLES && k < cap; ++k) {
    const VSpace& q = p->sp[k / NVROLES];
    variants[k] = q.on ? q.variant[k % NVROLES] : -1;
  }
  return ok();
}

ft_status funnel_volume_set_variant(ft_volume_plan* p, int32_t role, int32_t variant) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (role < 0 || role >= kVSpaces * NVROLES)
    return fail(FT_ERR_INVALID_ARG, "role must be in 0..%d (got %d)", kVSpaces * NVROLES - 1, role);
  const int si = role / NVROLES, r = role % NVROLES;
  if (!p->sp[si].on) return fail(FT_ERR_INVALID_ARG, "role %d belongs to a space the plan does not compute", role);
  if (variant < 0 || variant >= funnel::kMaxVariants || !(vrole_mask(p, si, r) & (1u << variant)))
    return fail(FT_ERR_INVALID_ARG, "%s has no kernel for variant %d", kVRoleName[si][r], variant);
  p->sp[si].variant[r] = variant;
  return ok();
}

ft_status funnel_volume_autotune(ft_volume_plan* p, void* stream, ft_tune_result* out, int32_t cap, int32_t* n) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (cap > 0 && !out) return fail(FT_ERR_INVALID_ARG, "out is NULL with cap > 0");
  ft_status st = check_volume_device(p);
  if (st != FT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t vb = (size_t)p->batch * p->vol_elems * sizeof(float);
  const size_t pb = (size_t)p->batch * p->param_elems * sizeof(float);
  void *a = nullptr, *b = nullptr, *w = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    (void)hipStreamSynchronize(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (w) (void)hipFree(w);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&a, vb) != hipSuccess || hipMalloc(&b, pb) != hipSuccess || hipMalloc(&w, p->ws_bytes) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_OUT_OF_MEMORY, "autotune scratch allocation failed");
  }
  if (hipMemsetAsync(a, 0, vb, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_HIP, "autotune set-up failed");
  }
  FtProfiler* saved = p->prof;
  p->prof = nullptr;
  int count = 0;
  // coordinate descent over the launches, two sweeps, each variant scored by
  // the whole forward chain (best of 5 after one warm-up)
  for (int sweep = 0; sweep < 2; ++sweep)
    for (int si = 0; si < kVSpaces; ++si) {
      if (!p->sp[si].on) continue;
      for (int r = 0; r < NVROLES; ++r) {
        const unsigned mask = vrole_mask(p, si, r);
        int& cur = p->sp[si].variant[r];
        float best = 1e30f, first_ms = -1.f;
        int best_v = cur, tried = 0;
        for (int v = 0; v < funnel::kMaxVariants; ++v) {
          if (!(mask & (1u << v))) continue;
          const int keep = cur;
          cur = v;
          float ms_min = 1e30f;
          hipError_t e = hipSuccess;
          for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess)
              e = enqueue_volume(p, static_cast<float*>(a), static_cast<float*>(b), static_cast<char*>(w), s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && rep > 0 && ms < ms_min) ms_min = ms;
          }
          cur = keep;
          if (e != hipSuccess) {
            p->prof = saved;
            cleanup();
            return hip_fail(e, "autotune launch");
          }
          if (v == keep) first_ms = ms_min;
          ++tried;
          if (ms_min < best) {
            best = ms_min;
            best_v = v;
          }
        }
        cur = best_v;
        if (sweep == 0) continue;
        if (count < cap) {
          std::memset(&out[count], 0, sizeof(ft_tune_result));
          std::snprintf(out[count].name, sizeof(out[count].name), "%s", kVRoleName[si][r]);
          out[count].variant = best_v;
          out[count].n_tried = tried;
          out[count].ms = best;
          out[count].ms_default = first_ms;
        }
        ++count;
      }
    }
  p->prof = saved;
  cleanup();
  if (n) *n = count < cap ? count : cap;
  return ok();
}

ft_status funnel_volume_profile_enable(ft_volume_plan* p, int32_t max_records) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  ft_status st = check_volume_device(p);
  if (st != FT_OK) return st;
  return profiler_enable(p->prof, max_records);
}

ft_status funnel_volume_profile_read(ft_volume_plan* p, ft_kernel_time* out, int32_t cap, int32_t* n) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  return profiler_read(p->prof, out, cap, n);
}

ft_status funnel_volume_profile_disable(ft_volume_plan* p) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  free_profiler(p->prof);
  p->prof = nullptr;
  return ok();
}

}  // extern "C"
