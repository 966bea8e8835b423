// funnel_api.cpp -- the C ABI declared in include/funnel.h: argument
// validation (host only, before any device work), plans with their FP64-derived
// twiddle tables, workspace layout and the order of the passes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/funnel.h"
#include "funnel_internal.hpp"

// Event pairs around each launch, filled while profiling is enabled.
struct FtProfiler {
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev0, ev1;
  std::vector<const char*> name;
  std::vector<double> bytes;
};

struct ft_plan {
  FtProfiler* prof;           // optional, owned
  int device;
  int batch, N, M, Np, h;
  int spaces;                 // FT_SPACE_* bits
  float2* tw;                 // device twiddle tables
  size_t tw_np, tw_m, tw_n;   // offsets (float2) of the tables for Np, M, N
  size_t plane_elems;         // floats of plane per image
  size_t off_inv_plane;       // floats from the image's plane block to the inverse plane
  size_t ws_bytes;            // forward / adjoint workspace
  size_t ws_off_inv;          // bytes from ws to the inverse-space spectrum
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

// exp(-i 2 pi m / L), m = 0 .. L-1, evaluated in double and rounded to float
void fill_twiddles(float2* dst, int L) {
  for (int m = 0; m < L; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)L;
    dst[m] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
}

// Run one launch, bracketed by events when the plan is being profiled.
template <class Fn>
hipError_t timed(const ft_plan* p, hipStream_t s, const char* name, double bytes, Fn&& fn) {
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
  if (d->precision != FT_PREC_FP32) return fail(FT_ERR_INVALID_ARG, "unknown precision %d", d->precision);
  if (d->flags != 0) return fail(FT_ERR_INVALID_ARG, "unknown plan flags 0x%x", d->flags);
  const long long N = d->rows, M = d->cols;
  long long Np = d->padded_len == 0 ? N + M : d->padded_len;
  if (d->padded_len < 0 || (Np & 1) || Np < N + M)
    return fail(FT_ERR_INVALID_ARG, "padded_len must be 0 or even and >= rows+cols (got %d)", d->padded_len);
  if (Np > (1 << 20) || M > (1 << 20) || N > (1 << 20))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "transform length too large");
  const bool reg = d->spaces & FT_SPACE_REGULAR, inv = d->spaces & FT_SPACE_INVERSE;
  if (!funnel::length_supported((int)Np))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for padded length %lld", Np);
  if (reg && !funnel::length_supported((int)M))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for row length %lld (image width)", M);
  if (inv && !funnel::length_supported((int)N))
    return fail(FT_ERR_UNSUPPORTED_SIZE, "no kernel for row length %lld (image height)", N);
  const long long h = Np / 2 - 1;
  const long long plane_elems = (reg ? Np * M : 0) + (inv ? Np * N : 0);
  if ((long long)d->batch * plane_elems > (1ll << 40))
    return fail(FT_ERR_INVALID_ARG, "batch too large");

  int dev = -1, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(FT_ERR_NO_DEVICE, "no HIP device");
  if (hipGetDevice(&dev) != hipSuccess) return fail(FT_ERR_NO_DEVICE, "no current HIP device");

  ft_plan* p = new (std::nothrow) ft_plan();
  if (!p) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->device = dev;
  p->batch = d->batch;
  p->N = (int)N;
  p->M = (int)M;
  p->Np = (int)Np;
  p->h = (int)h;
  p->spaces = d->spaces;
  p->plane_elems = (size_t)plane_elems;
  p->off_inv_plane = reg ? (size_t)(Np * M) : 0;
  const size_t s_reg = reg ? align_up((size_t)d->batch * h * M * sizeof(float2), 256) : 0;
  const size_t s_inv = inv ? align_up((size_t)d->batch * h * N * sizeof(float2), 256) : 0;
  p->ws_off_inv = s_reg;
  p->ws_bytes = s_reg + s_inv;

  // twiddle tables for Np, M and N, back to back
  p->tw_np = 0;
  p->tw_m = (size_t)Np;
  p->tw_n = p->tw_m + (size_t)M;
  const size_t ntw = p->tw_n + (size_t)N;
  float2* host = new (std::nothrow) float2[ntw];
  if (!host) {
    delete p;
    return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  fill_twiddles(host + p->tw_np, (int)Np);
  fill_twiddles(host + p->tw_m, (int)M);
  fill_twiddles(host + p->tw_n, (int)N);
  hipError_t e = hipMalloc(&p->tw, ntw * sizeof(float2));
  if (e != hipSuccess) {
    delete[] host;
    delete p;
    return fail(FT_ERR_OUT_OF_MEMORY, "hipMalloc of twiddle tables: %s", hipGetErrorString(e));
  }
  e = hipMemcpy(p->tw, host, ntw * sizeof(float2), hipMemcpyHostToDevice);
  delete[] host;
  if (e != hipSuccess) {
    (void)hipFree(p->tw);
    delete p;
    return hip_fail(e, "hipMemcpy of twiddle tables");
  }
  *out = p;
  return ok();
}

void funnel_plan_destroy(ft_plan* p) {
  if (!p) return;
  free_profiler(p->prof);
  if (p->tw) (void)hipFree(p->tw);
  delete p;
}

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

ft_status funnel_padded_len(const ft_plan* p, int32_t* np) {
  if (!p || !np) return fail(FT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  *np = p->Np;
  return ok();
}

static ft_status check_call(const ft_plan* p, const void* a, const void* b, const void* ws, size_t ws_bytes) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!a || !b || !ws) return fail(FT_ERR_INVALID_ARG, "input, output and workspace must be non-NULL");
  if (!aligned16(a) || !aligned16(b) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  if (ws_bytes < p->ws_bytes)
    return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, p->ws_bytes);
  return FT_OK;
}

ft_status funnel_forward(const ft_plan* p, const float* images, float* planes, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, images, planes, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = p->batch, N = p->N, M = p->M, Np = p->Np, h = p->h;
  const long long img = (long long)N * M, pst = (long long)p->plane_elems;
  char* w = static_cast<char*>(ws);
  const float2* tw_np = p->tw + p->tw_np;
  hipError_t e = hipSuccess;
  const double b = B;
  if (p->spaces & FT_SPACE_REGULAR) {
    float2* S = reinterpret_cast<float2*>(w);
    const long long sst = (long long)h * M;
    // pass A: columns of the image, (Np-N)/2 zero rows above
    e = timed(p, s, "fwd.regular.A", b * (4.0 * N * M + 8.0 * h * M), [&] {
      return funnel::launch_r2c(Np, false, images, S, M, N, (Np - N) / 2, img, sst, 1.0f, tw_np, B, s);
    });
    if (e == hipSuccess)
      e = timed(p, s, "fwd.regular.B", b * 16.0 * h * M,
                [&] { return funnel::launch_row(M, false, S, Np, h, sst, p->tw + p->tw_m, B, s); });
    if (e == hipSuccess)
      e = timed(p, s, "fwd.regular.C", b * (8.0 * h * M + 4.0 * Np * M), [&] {
        return funnel::launch_c2r(Np, false, false, S, planes, M, 0, Np, sst, pst, 1.0f / Np, tw_np, B, s);
      });
  }
  if (e == hipSuccess && (p->spaces & FT_SPACE_INVERSE)) {
    float2* S = reinterpret_cast<float2*>(w + p->ws_off_inv);
    const long long sst = (long long)h * N;
    // pass A of the dual form: rows of the image, (Np-M)/2 zero columns on the left
    e = timed(p, s, "fwd.inverse.A", b * (4.0 * N * M + 8.0 * h * N), [&] {
      return funnel::launch_r2c(Np, true, images, S, N, M, (Np - M) / 2, img, sst, 1.0f, tw_np, B, s);
    });
    if (e == hipSuccess)
      e = timed(p, s, "fwd.inverse.B", b * 16.0 * h * N,
                [&] { return funnel::launch_row(N, false, S, Np, h, sst, p->tw + p->tw_n, B, s); });
    if (e == hipSuccess)
      e = timed(p, s, "fwd.inverse.C", b * (8.0 * h * N + 4.0 * Np * N), [&] {
        return funnel::launch_c2r(Np, false, false, S, planes + p->off_inv_plane, N, 0, Np, sst, pst, 1.0f / Np,
                                  tw_np, B, s);
      });
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_adjoint(const ft_plan* p, const float* d_planes, float* d_images, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, d_planes, d_images, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int B = p->batch, N = p->N, M = p->M, Np = p->Np, h = p->h;
  const long long img = (long long)N * M, pst = (long long)p->plane_elems;
  char* w = static_cast<char*>(ws);
  const float2* tw_np = p->tw + p->tw_np;
  hipError_t e = hipSuccess;
  const bool reg = p->spaces & FT_SPACE_REGULAR;
  const double b = B;
  if (reg) {
    float2* S = reinterpret_cast<float2*>(w);
    const long long sst = (long long)h * M;
    // C^T: (2/Np) DFT along y of every plane column, rows 1..h
    e = timed(p, s, "adj.regular.Ct", b * (4.0 * Np * M + 8.0 * h * M), [&] {
      return funnel::launch_r2c(Np, false, d_planes, S, M, Np, 0, pst, sst, 2.0f / Np, tw_np, B, s);
    });
    // B^T: conjugate DFT along x', transposed interpolation
    if (e == hipSuccess)
      e = timed(p, s, "adj.regular.Bt", b * 16.0 * h * M,
                [&] { return funnel::launch_row(M, true, S, Np, h, sst, p->tw + p->tw_m, B, s); });
    // A^T: Re of the conjugate y DFT, image rows only
    if (e == hipSuccess)
      e = timed(p, s, "adj.regular.At", b * (8.0 * h * M + 4.0 * N * M), [&] {
        return funnel::launch_c2r(Np, false, false, S, d_images, M, (Np - N) / 2, N, sst, img, 0.5f, tw_np, B, s);
      });
  }
  if (e == hipSuccess && (p->spaces & FT_SPACE_INVERSE)) {
    float2* S = reinterpret_cast<float2*>(w + p->ws_off_inv);
    const long long sst = (long long)h * N;
    e = timed(p, s, "adj.inverse.Ct", b * (4.0 * Np * N + 8.0 * h * N), [&] {
      return funnel::launch_r2c(Np, false, d_planes + p->off_inv_plane, S, N, Np, 0, pst, sst, 2.0f / Np, tw_np, B,
                                s);
    });
    if (e == hipSuccess)
      e = timed(p, s, "adj.inverse.Bt", b * 16.0 * h * N,
                [&] { return funnel::launch_row(N, true, S, Np, h, sst, p->tw + p->tw_n, B, s); });
    // transposed write into the image rows; adds to the regular space's result
    if (e == hipSuccess)
      e = timed(p, s, "adj.inverse.At", b * (8.0 * h * N + (reg ? 8.0 : 4.0) * N * M), [&] {
        return funnel::launch_c2r(Np, true, reg, S, d_images, N, (Np - M) / 2, M, sst, img, 0.5f, tw_np, B, s);
      });
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

ft_status funnel_profile_enable(ft_plan* p, int32_t max_records) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (max_records < 1 || max_records > (1 << 20))
    return fail(FT_ERR_INVALID_ARG, "max_records must be in 1..2^20 (got %d)", max_records);
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  FtProfiler* pr = new (std::nothrow) FtProfiler();
  if (!pr) return fail(FT_ERR_OUT_OF_MEMORY, "host allocation failed");
  pr->cap = max_records;
  pr->ev0.resize(max_records);
  pr->ev1.resize(max_records);
  pr->name.assign(max_records, nullptr);
  pr->bytes.assign(max_records, 0.0);
  for (int i = 0; i < max_records; ++i) {
    if (hipEventCreate(&pr->ev0[i]) != hipSuccess || hipEventCreate(&pr->ev1[i]) != hipSuccess) {
      pr->ev0.resize(i);
      pr->ev1.resize(i);
      free_profiler(pr);
      return fail(FT_ERR_HIP, "hipEventCreate failed");
    }
  }
  free_profiler(p->prof);
  p->prof = pr;
  return ok();
}

ft_status funnel_profile_read(ft_plan* p, ft_kernel_time* out, int32_t cap, int32_t* n) {
  if (!p || !out || !n || cap < 1) return fail(FT_ERR_INVALID_ARG, "plan, out and n must be non-NULL, cap >= 1");
  FtProfiler* pr = p->prof;
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
    while (k < cnt && std::strcmp(out[k].name, pr->name[i]) != 0) ++k;
    if (k == cnt) {
      if (cnt == cap) continue;
      std::memset(&out[k], 0, sizeof(ft_kernel_time));
      std::snprintf(out[k].name, sizeof(out[k].name), "%s", pr->name[i]);
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

ft_status funnel_profile_disable(ft_plan* p) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  free_profiler(p->prof);
  p->prof = nullptr;
  return ok();
}

ft_status funnel_peaks_workspace_size(const ft_plan* p, int32_t K, size_t* bytes) {
  if (!p || !bytes) return fail(FT_ERR_INVALID_ARG, "plan and bytes must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  const int ns = (p->spaces == FT_SPACE_BOTH) ? 2 : 1;
  int tiles = 0;
  if (p->spaces & FT_SPACE_REGULAR) tiles = funnel::peaks_tiles(p->Np, p->M);
  if (p->spaces & FT_SPACE_INVERSE) {
    const int t = funnel::peaks_tiles(p->Np, p->N);
    tiles = t > tiles ? t : tiles;
  }
  *bytes = funnel::peaks_workspace_bytes(p->batch * ns, tiles, K);
  return ok();
}

ft_status funnel_peaks(const ft_plan* p, const float* planes, int32_t K, float threshold, int32_t radius,
                       uint32_t flags, ft_peak* peaks, int32_t* n_found, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (!planes || !peaks || !n_found || !ws) return fail(FT_ERR_INVALID_ARG, "pointers must be non-NULL");
  if (K < 1 || K > 256) return fail(FT_ERR_INVALID_ARG, "K must be in 1..256 (got %d)", K);
  if (radius < 1 || radius > 8) return fail(FT_ERR_INVALID_ARG, "radius must be in 1..8 (got %d)", radius);
  if (std::isnan(threshold)) return fail(FT_ERR_INVALID_ARG, "threshold is NaN");
  if (flags & ~(uint32_t)(FT_PEAK_CLAMP_BORDER | FT_PEAK_KEEP_PAD_BOUNDARY))
    return fail(FT_ERR_INVALID_ARG, "unknown peak flags 0x%x", flags);
  if (!aligned16(planes) || !aligned16(peaks) || !aligned16(n_found) || !aligned16(ws))
    return fail(FT_ERR_MISALIGNED, "device pointers must be 16-byte aligned");
  size_t need = 0;
  ft_status st = funnel_peaks_workspace_size(p, K, &need);
  if (st != FT_OK) return st;
  if (ws_bytes < need) return fail(FT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
  if ((st = check_device(p)) != FT_OK) return st;
  (void)hipGetLastError();
  int rows[2], cols[2], himg[2];
  long long off[2];
  int ns = 0;
  if (p->spaces & FT_SPACE_REGULAR) {
    rows[ns] = p->Np; cols[ns] = p->M; himg[ns] = p->N; off[ns] = 0; ++ns;
  }
  if (p->spaces & FT_SPACE_INVERSE) {
    rows[ns] = p->Np; cols[ns] = p->N; himg[ns] = p->M; off[ns] = (long long)p->off_inv_plane; ++ns;
  }
  hipError_t e = funnel::launch_peaks(planes, (long long)p->plane_elems, p->batch, ns, rows, cols, himg, off, K,
                                      threshold, radius, (flags & FT_PEAK_CLAMP_BORDER) ? 0 : 1,
                                      (flags & FT_PEAK_KEEP_PAD_BOUNDARY) ? 1 : 0, peaks, n_found, ws,
                                      static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return ok();
}

}  // extern "C"
