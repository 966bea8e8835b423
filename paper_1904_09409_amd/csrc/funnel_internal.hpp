// funnel_internal.hpp -- launchers shared between the kernel and API units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <type_traits>

#include "../../include/funnel.h"

namespace funnel {

// Where image i's input and output start (elements): uniform strides, or
// per-image offset tables in device memory (ragged batches).
struct ImgMap {
  long long in_stride, out_stride;
  const long long* in_off;
  const long long* out_off;
  __host__ __device__ long long in(int i) const { return in_off ? in_off[i] : (long long)i * in_stride; }
  __host__ __device__ long long out(int i) const { return out_off ? out_off[i] : (long long)i * out_stride; }
};

// arithmetic of the DFT passes: FP32 butterflies, or matrix-core products
// with BF16 / FP16 hi + lo operands and FP32 accumulation (same values as
// FT_PREC_* in funnel.h)
enum Prec : int { kPrecFP32 = 0, kPrecBF16x3 = 1, kPrecFP16x3 = 2 };

bool length_supported(int L);

// bit v set: tile variant v has a kernel for this length and precision
// (register-resident tiles first, then the LDS-resident ones for FP32; split
// precisions: 0 when the length has no matrix-core kernel)
unsigned col_variant_mask(int L, int prec);
unsigned row_variant_mask(int M, int prec);
// (bits 0-7: register tiles, 8-10: LDS-resident tiles)
constexpr int kMaxVariants = 12;

// real lines (zero-padded to L) -> half spectrum rows 1..L/2-1, times scale*(-1)^k
hipError_t launch_r2c(int L, int variant, int prec, bool trans, const float* in, float2* out, int nlines, int lin, int off,
                      ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);

// half spectrum rows 1..L/2-1 -> real lines, rows [r0, r0+nout) stored (or added)
hipError_t launch_c2r(int L, int variant, int prec, bool trans, bool accum, const float2* in, float* out, int nlines, int r0,
                      int nout, ImgMap map, float scale, const float2* tw, int batch, hipStream_t s);

// per frequency row (rpf data rows each, sharing that row's ratio s): NVMT
// gather + DFT along x' (forward) or its transpose (adjoint), in place
hipError_t launch_row(int M, int variant, int prec, bool adj, float2* data, int Lp, int h, int rpf, long long img_stride, const float2* tw,
                      int batch, hipStream_t s);

// per frequency row: band-limited (chirp-z) NVMT fused with the DFT along x'
// (forward) or its conjugate transpose (adjoint), in place, for row length W.
// cz: [h][2W] chirp spectra (s / 2W) DFT_2W(c'), wz: [h][W] chirps
// exp(-j pi s x^2 / W), tw: twiddles of length 2W.  Bit v of the mask set:
// tile variant v has a kernel for W (0: no chirp-z kernel for this length).
unsigned chirp_variant_mask(int W);
hipError_t launch_chirp(int W, int variant, bool adj, float2* data, int h, long long img_stride, const float2* cz,
                        const float2* wz, const float2* tw, int batch, hipStream_t s);
// host: the FP64-derived tables above for rows n2 = 1..h of padded length Np
void chirp_tables(int W, int Np, int h, float2* cz, float2* wz);

// Sub-cell refinement of peaks (uniform plans, power-of-two row lengths).
// launch_row_idft: rows G -> g (inverse x' DFT, centred, 1/W) in place.
// launch_refine_init: iteration state from the peak lists.
// launch_refine_iter: one iteration (final = 0) or the evaluation and the
// records (final = 1) for space index s of the plan.
bool refine_length_supported(int W);
size_t refine_state_bytes();
// launch_row_lerp: spectrum rows S -> g by the linear NVMT alone (the row
// pass without its DFT), in place; rows n2 = 1 .. h, padded length Lp.
hipError_t launch_row_lerp(int W, float2* data, int h, int Lp, long long img_stride, int batch, hipStream_t s);
hipError_t launch_row_idft(int W, float2* data, int h, long long img_stride, const float2* tw, int batch,
                           hipStream_t s);
hipError_t launch_refine_init(const ft_peak* peaks, const int32_t* n_found, int batch, int ns, int K, int W0, int W1,
                              int Np, void* state, hipStream_t s);
hipError_t launch_refine_iter(const float2* g, long long img_stride, int h, int W, int s, int ns, int K, int batch,
                              const int32_t* n_found, void* state, float2* A, int Np, int space_id, int N, int M,
                              int final, ft_refined* out, hipStream_t st);

// Volumes (App. A).  The y' pass: per slice n3 (h of them, ratio 2 n3 / Lz)
// and column of data [h][L][nx] (per volume, vol_stride complex apart),
// linear-interpolation gather along y fused with the centred DFT along y', in
// place.  ycol_lines: columns per block of a variant.
unsigned ycol_variant_mask(int L);
int ycol_lines(int variant);
hipError_t launch_ycol(int L, int variant, float2* data, int Lz, int h, int nx, long long vol_stride,
                       const float2* tw, int batch, hipStream_t s);
// slices [ny][nx] -> [nx][ny], `slices` of them back to back
hipError_t launch_transpose_slices(const float* in, float* out, int slices, int ny, int nx, hipStream_t s);
// 3D peaks of the parameter volumes [batch][nz][ny][nx] (stride floats apart);
// zimg: depth of the transformed volume (the faces of its expansion).
// Records and counts go to peaks[(v * ns + sp) * K ..] and n_found[v * ns + sp],
// each record tagged with space_id.
int vpeaks_tiles(int nz, int ny, int nx);
size_t vpeaks_workspace_bytes(int nvol, int tiles, int K);
hipError_t launch_vpeaks(const float* params, long long stride, int batch, int nz, int ny, int nx, int zimg, int K,
                         float thr, int radius, int wrap, int keep_border, int ns, int sp, int space_id,
                         ft_plane_peak* peaks, int32_t* n_found, void* ws, hipStream_t s);

size_t peaks_workspace_bytes(int nplanes_total, int tiles, int K);
int peaks_tiles(int rows, int cols);
hipError_t launch_peaks(const float* planes, ImgMap map, const int* gidx, int batch, int nspaces, int space0,
                        const int* rows, const int* cols, const int* himg, const long long* offset, int K, float thr,
                        int radius, int wrap, int keep_border, ft_peak* peaks, int32_t* n_found, void* ws,
                        hipStream_t s);

// Sec. 4.5 line verification of the peak lists written by launch_peaks, for
// the images of one size class (N x M, offsets by map.in, caller indices by
// gidx): one record per peak slot, [image][space][K]
hipError_t launch_verify(const float* images, ImgMap map, const int* gidx, int count, int ns, int N, int M,
                         const ft_peak* peaks, const int32_t* n_found, int K, int D, float min_contrast,
                         int min_length, ft_line_check* out, hipStream_t s);

}  // namespace funnel
