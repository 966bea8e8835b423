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
  int variant[12];            // tile variant of each pass launch (see Role)
};

// The twelve kernel launches: three passes per space, forward and adjoint.
enum Role {
  FA_REG, FB_REG, FC_REG, FA_INV, FB_INV, FC_INV,
  AC_REG, AB_REG, AA_REG, AC_INV, AB_INV, AA_INV, NROLES
};
static const char* const kRoleName[NROLES] = {
    "fwd.regular.A", "fwd.regular.B", "fwd.regular.C", "fwd.inverse.A", "fwd.inverse.B", "fwd.inverse.C",
    "adj.regular.Ct", "adj.regular.Bt", "adj.regular.At", "adj.inverse.Ct", "adj.inverse.Bt", "adj.inverse.At"};

static bool role_is_row(int r) { return r == FB_REG || r == FB_INV || r == AB_REG || r == AB_INV; }
static bool role_regular(int r) { return r <= FC_REG || (r >= AC_REG && r <= AA_REG); }
static bool role_active(const ft_plan* p, int r) {
  return (p->spaces & (role_regular(r) ? FT_SPACE_REGULAR : FT_SPACE_INVERSE)) != 0;
}
static unsigned role_mask(const ft_plan* p, int r) {
  if (!role_is_row(r)) return funnel::col_variant_mask(p->Np);
  return funnel::row_variant_mask(role_regular(r) ? p->M : p->N);
}


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

  // default tile variants: the lowest-numbered one each kernel has
  for (int r = 0; r < NROLES; ++r) {
    const unsigned m = role_mask(p, r);
    p->variant[r] = 0;
    for (int v = 0; v < funnel::kMaxVariants; ++v)
      if (m & (1u << v)) { p->variant[r] = v; break; }
  }

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

// Algorithmic HBM bytes of one launch: each input read once, each output
// written once (a read-modify-write output counts twice).
static double role_bytes(const ft_plan* p, int r) {
  const double B = p->batch, N = p->N, M = p->M, Np = p->Np, h = p->h;
  const double W = role_regular(r) ? M : N;  // lines of the spectrum
  switch (r) {
    case FA_REG: case FA_INV: return B * (4.0 * N * M + 8.0 * h * W);
    case FB_REG: case FB_INV: case AB_REG: case AB_INV: return B * 16.0 * h * W;
    case FC_REG: case FC_INV: return B * (8.0 * h * W + 4.0 * Np * W);
    case AC_REG: case AC_INV: return B * (4.0 * Np * W + 8.0 * h * W);
    case AA_REG: return B * (8.0 * h * M + 4.0 * N * M);
    case AA_INV: return B * (8.0 * h * N + ((p->spaces & FT_SPACE_REGULAR) ? 8.0 : 4.0) * N * M);
  }
  return 0.0;
}

// One pass launch.  src: images (forward) or plane gradients (adjoint);
// dst: planes (forward) or image gradients (adjoint).
static hipError_t run_role(const ft_plan* p, int r, int v, const float* src, float* dst, char* w, hipStream_t s) {
  const int B = p->batch, N = p->N, M = p->M, Np = p->Np, h = p->h;
  const long long img = (long long)N * M, pst = (long long)p->plane_elems;
  const float2* tw_np = p->tw + p->tw_np;
  float2* Sr = reinterpret_cast<float2*>(w);
  float2* Si = reinterpret_cast<float2*>(w + p->ws_off_inv);
  const long long sr = (long long)h * M, si = (long long)h * N;
  const bool reg = p->spaces & FT_SPACE_REGULAR;
  switch (r) {
    // forward, regular space: y DFT of the image columns on the expanded frame,
    // NVMT + x' DFT per frequency row, Hermitian inverse y DFT
    case FA_REG: return funnel::launch_r2c(Np, v, false, src, Sr, M, N, (Np - N) / 2, img, sr, 1.0f, tw_np, B, s);
    case FB_REG: return funnel::launch_row(M, v, false, Sr, Np, h, sr, p->tw + p->tw_m, B, s);
    case FC_REG:
      return funnel::launch_c2r(Np, v, false, false, Sr, dst, M, 0, Np, sr, pst, 1.0f / Np, tw_np, B, s);
    // forward, inverse space: the same on the transposed image (rows read directly)
    case FA_INV: return funnel::launch_r2c(Np, v, true, src, Si, N, M, (Np - M) / 2, img, si, 1.0f, tw_np, B, s);
    case FB_INV: return funnel::launch_row(N, v, false, Si, Np, h, si, p->tw + p->tw_n, B, s);
    case FC_INV:
      return funnel::launch_c2r(Np, v, false, false, Si, dst + p->off_inv_plane, N, 0, Np, si, pst, 1.0f / Np,
                                tw_np, B, s);
    // adjoint, regular space: (2/Np) y DFT of the plane columns, conjugate x'
    // DFT + transposed interpolation, real part of the conjugate y DFT cropped
    case AC_REG: return funnel::launch_r2c(Np, v, false, src, Sr, M, Np, 0, pst, sr, 2.0f / Np, tw_np, B, s);
    case AB_REG: return funnel::launch_row(M, v, true, Sr, Np, h, sr, p->tw + p->tw_m, B, s);
    case AA_REG:
      return funnel::launch_c2r(Np, v, false, false, Sr, dst, M, (Np - N) / 2, N, sr, img, 0.5f, tw_np, B, s);
    // adjoint, inverse space: transposed write into the image rows, added to
    // the regular space's result when both spaces are computed
    case AC_INV:
      return funnel::launch_r2c(Np, v, false, src + p->off_inv_plane, Si, N, Np, 0, pst, si, 2.0f / Np, tw_np, B,
                                s);
    case AB_INV: return funnel::launch_row(N, v, true, Si, Np, h, si, p->tw + p->tw_n, B, s);
    case AA_INV:
      return funnel::launch_c2r(Np, v, true, reg, Si, dst, N, (Np - M) / 2, M, si, img, 0.5f, tw_np, B, s);
  }
  return hipErrorInvalidValue;
}

static ft_status run_roles(const ft_plan* p, int first, int last, const float* src, float* dst, void* ws,
                           hipStream_t s) {
  (void)hipGetLastError();
  char* w = static_cast<char*>(ws);
  for (int r = first; r <= last; ++r) {
    if (!role_active(p, r)) continue;
    hipError_t e = timed(p, s, kRoleName[r], role_bytes(p, r),
                         [&] { return run_role(p, r, p->variant[r], src, dst, w, s); });
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return ok();
}

ft_status funnel_forward(const ft_plan* p, const float* images, float* planes, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, images, planes, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  return run_roles(p, FA_REG, FC_INV, images, planes, ws, static_cast<hipStream_t>(stream));
}

ft_status funnel_adjoint(const ft_plan* p, const float* d_planes, float* d_images, void* ws, size_t ws_bytes,
                         void* stream) {
  ft_status st = check_call(p, d_planes, d_images, ws, ws_bytes);
  if (st != FT_OK) return st;
  if ((st = check_device(p)) != FT_OK) return st;
  return run_roles(p, AC_REG, AA_INV, d_planes, d_images, ws, static_cast<hipStream_t>(stream));
}

ft_status funnel_autotune(ft_plan* p, void* stream, ft_tune_result* out, int32_t cap, int32_t* n) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (cap < 0 || (cap > 0 && (!out || !n))) return fail(FT_ERR_INVALID_ARG, "bad result buffer");
  ft_status st = check_device(p);
  if (st != FT_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t img_bytes = (size_t)p->batch * p->N * p->M * sizeof(float);
  const size_t pl_bytes = (size_t)p->batch * p->plane_elems * sizeof(float);
  void *a = nullptr, *b = nullptr, *w = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&] {
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (w) (void)hipFree(w);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  // a holds images or plane gradients, b planes or image gradients: size both for the larger
  const size_t big = img_bytes > pl_bytes ? img_bytes : pl_bytes;
  if (hipMalloc(&a, big) != hipSuccess || hipMalloc(&b, big) != hipSuccess ||
      hipMalloc(&w, p->ws_bytes ? p->ws_bytes : 256) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_OUT_OF_MEMORY, "autotune scratch allocation failed");
  }
  if (hipMemsetAsync(a, 0, big, s) != hipSuccess || hipMemsetAsync(b, 0, big, s) != hipSuccess ||
      hipMemsetAsync(w, 0, p->ws_bytes ? p->ws_bytes : 256, s) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(FT_ERR_HIP, "autotune set-up failed");
  }
  FtProfiler* saved = p->prof;
  p->prof = nullptr;
  int count = 0;
  for (int r = 0; r < NROLES; ++r) {
    if (!role_active(p, r)) continue;
    const unsigned mask = role_mask(p, r);
    float best = 1e30f, first_ms = -1.f;
    int best_v = p->variant[r], tried = 0;
    for (int v = 0; v < funnel::kMaxVariants; ++v) {
      if (!(mask & (1u << v))) continue;
      float ms_min = 1e30f;
      hipError_t e = hipSuccess;
      for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = run_role(p, r, v, static_cast<float*>(a), static_cast<float*>(b),
                                          static_cast<char*>(w), s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && rep > 0 && ms < ms_min) ms_min = ms;
      }
      if (e != hipSuccess) {
        p->prof = saved;
        cleanup();
        return hip_fail(e, "autotune launch");
      }
      if (v == p->variant[r]) first_ms = ms_min;
      ++tried;
      if (ms_min < best) {
        best = ms_min;
        best_v = v;
      }
    }
    p->variant[r] = best_v;
    if (count < cap) {
      std::memset(&out[count], 0, sizeof(ft_tune_result));
      std::snprintf(out[count].name, sizeof(out[count].name), "%s", kRoleName[r]);
      out[count].variant = best_v;
      out[count].n_tried = tried;
      out[count].ms = best;
      out[count].ms_default = first_ms;
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
  for (int r = 0; r < NROLES && r < cap; ++r) variants[r] = role_active(p, r) ? p->variant[r] : -1;
  return ok();
}

ft_status funnel_plan_set_variant(ft_plan* p, int32_t role, int32_t variant) {
  if (!p) return fail(FT_ERR_INVALID_ARG, "plan is NULL");
  if (role < 0 || role >= NROLES) return fail(FT_ERR_INVALID_ARG, "role must be in 0..%d", NROLES - 1);
  if (variant < 0 || variant >= funnel::kMaxVariants || !(role_mask(p, role) & (1u << variant)))
    return fail(FT_ERR_INVALID_ARG, "variant %d has no kernel for role %s", variant, kRoleName[role]);
  p->variant[role] = variant;
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
