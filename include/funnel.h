/*
 * funnel.h -- C ABI of the MI355X (gfx950) funnel-transform library.
 *
 * The funnel transform (Wei, Feng, Zheng, "Funnel Transform for Straight Line
 * Detection", arXiv 1904.09409) maps a grayscale image to a slope-intercept
 * parameter plane in which every straight line focuses to a peak.  It is three
 * 1D Fourier transforms around the nonlinear variable-metric transform (NVMT),
 * Sec. 3.1:
 *
 *   S(x, w2)   = DFT_y  of the expanded image            (Sec. 3.1 step 1, Sec. 4.2)
 *   g(x', w2)  = S(x'/s, w2), s = w2/w_max               (step 2, Eq. 17; linear
 *                                                          interpolation, Sec. V)
 *   G(w1, w2)  = DFT_x' of g                             (step 3)
 *   P(w1, y)   = inverse DFT_w2 of G                     (step 4, Eq. 19)
 *
 * The regular space covers slopes in (-1, 1]; the inverse space is the same
 * transform of the transposed image and covers the steeper lines (Sec. 4.1,
 * Sec. 4.2).  Peaks of |P| are found by the list rule of Sec. 4.4 and read as
 * line parameters by Eqs. 22-25.
 *
 * Conventions fixed by this library (the paper leaves them open):
 *   - image I[r][c]: N rows (height), M columns (width), row-major float32,
 *     N and M even and >= 4; images of a batch are contiguous (stride N*M).
 *   - expansion (Sec. 4.2): the y axis is padded to Np = N+M (or padded_len)
 *     with (Np-N)/2 zero rows on top; the frame centre is the origin:
 *     y = r' - Np/2, x = c - M/2.
 *   - w_max = pi, hence s = 2 n2 / Np for frequency row n2 = 1 .. Np/2-1; the
 *     DC and Nyquist rows are zero and negative rows follow by conjugate
 *     symmetry (Sec. 3.1).
 *   - NVMT: g[x'] = (1-t) f[i0] + t f[i0+1], i0 = floor((x' Np + M n2)/(2 n2))
 *     by exact integer division, f = S row indexed from 0 at x = -M/2, zero
 *     outside [0, M).
 *   - forward DFTs unnormalised; the last inverse DFT carries 1/Np.
 *   - regular plane: float32 P[Np][M], row = y + Np/2, column = m1 + M/2; a
 *     line row = k*col + b focuses at m1 = -k M/2, y = b + k M/2 - N/2.
 *     Inverse plane: float32 P_inv[Np][N], the same for the transposed image.
 *   - the planes of one image are contiguous: regular first, then inverse
 *     (for the spaces the plan computes); images follow each other with the
 *     stride given by funnel_plane_elems().
 *
 * Ownership and threading: the caller owns every image, plane, peak and
 * workspace buffer (device memory).  A plan owns only its constant tables.
 * funnel_forward / funnel_adjoint / funnel_peaks never allocate, never
 * synchronise and never print: they enqueue kernels on the given stream and
 * return.  Plans are immutable after creation and may be used from several
 * streams at once if every concurrent call gets its own workspace.
 *
 * Errors: every call validates its arguments on the host before any device
 * work; on error it returns a status, writes nothing and keeps a message for
 * funnel_last_error() (thread-local).  Device pointers must be 16-byte
 * aligned.  Faults of already-enqueued kernels surface as FT_ERR_HIP from a
 * later call or from the caller's stream synchronisation.
 */
#ifndef FUNNEL_H
#define FUNNEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FT_OK = 0,
  FT_ERR_INVALID_ARG = 1,       /* NULL pointer, bad count, bad flag, NaN threshold ... */
  FT_ERR_UNSUPPORTED_SIZE = 2,  /* a transform length this build has no kernel for */
  FT_ERR_MISALIGNED = 3,        /* a device pointer not 16-byte aligned */
  FT_ERR_WORKSPACE_TOO_SMALL = 4,
  FT_ERR_NO_DEVICE = 5,         /* no HIP device, or the plan's device is not current */
  FT_ERR_HIP = 6,               /* a HIP runtime call failed */
  FT_ERR_OUT_OF_MEMORY = 7      /* plan creation could not allocate its tables */
} ft_status;

/* Which parameter spaces a plan computes (Sec. 4.1). */
enum { FT_SPACE_REGULAR = 1, FT_SPACE_INVERSE = 2, FT_SPACE_BOTH = 3 };

/* Arithmetic of the DFT stages.
 *   FT_PREC_FP32   : FP32 butterflies (the reference path).
 *   FT_PREC_BF16X3 : every radix-16 / radix-8 DFT stage as a matrix-core
 *                    product with split operands, X = X_hi + X_lo and
 *                    W = W_hi + W_lo in BF16, keeping the three products
 *                    hi*hi + hi*lo + lo*hi, FP32 accumulation.
 *   FT_PREC_FP16X3 : the same in FP16, operands scaled per butterfly by a
 *                    power of two.
 * Twiddle factors, the NVMT coordinates and weights, and all data between
 * stages stay FP32 in every mode.  The split precisions need power-of-two
 * lengths: Np in 128 .. 4096 and the row lengths (M, and N for the inverse
 * space) in 64 .. 4096; other shapes give FT_ERR_UNSUPPORTED_SIZE. */
enum { FT_PREC_FP32 = 0, FT_PREC_BF16X3 = 1, FT_PREC_FP16X3 = 2 };

/* ft_plan_desc flags.
 *   FT_PLAN_NVMT_CHIRPZ : realise the NVMT by band-limited (chirp-z)
 *     resampling, the way the paper adopts at the opening of Sec. IV, instead
 *     of linear interpolation (Sec. V's O(M^2) option, the default).  Each
 *     frequency row n2 (ratio s = 2 n2 / Np) then gets, fused with the DFT
 *     along x', G[m1] = s sum_x S[x] exp(-j 2 pi s m1 x / W) over centred x
 *     and m1 in [-W/2, W/2), W = M (regular space) or N (inverse space): the
 *     resampled row's spectrum without interpolation attenuation.  It is
 *     computed by Bluestein's algorithm with FFTs of length 2W; the plan holds
 *     FP64-derived chirp tables of 24 * (Np/2 - 1) * W bytes per space.
 *     FP32 only; row lengths W must be powers of two in 64 .. 2048, else
 *     FT_ERR_UNSUPPORTED_SIZE.  Ragged plans use linear interpolation. */
enum { FT_PLAN_NVMT_CHIRPZ = 1u };

/* funnel_peaks flags. */
enum {
  FT_PEAK_CLAMP_BORDER = 1u,     /* neighbourhood clamped at the plane edge instead of wrapping */
  FT_PEAK_KEEP_PAD_BOUNDARY = 2u /* do not drop the cells where the expansion borders focus */
};

typedef struct ft_plan ft_plan;

typedef struct {
  int32_t batch;       /* number of images, >= 1 */
  int32_t rows;        /* N, image height, even, >= 4 */
  int32_t cols;        /* M, image width, even, >= 4 */
  int32_t padded_len;  /* Np; 0 means N+M (Sec. 4.2); else even and >= N+M */
  int32_t spaces;      /* FT_SPACE_REGULAR, FT_SPACE_INVERSE or FT_SPACE_BOTH */
  int32_t precision;   /* FT_PREC_FP32, FT_PREC_BF16X3 or FT_PREC_FP16X3 */
  uint32_t flags;      /* 0 or FT_PLAN_NVMT_CHIRPZ */
} ft_plan_desc;

/* One detected peak (Sec. 4.4) and its line (Eqs. 22-25).
 * space 0 (regular): the line is row = slope*col + intercept;
 * space 1 (inverse): the line is col = slope*row + intercept
 * (pixel-index coordinates of the input image, pixel centres at integers). */
typedef struct {
  int32_t image;
  int32_t space;
  int32_t row;         /* plane row (intercept bin) */
  int32_t col;         /* plane column (slope bin) */
  float value;         /* brightness |P| */
  float slope;
  float intercept;
} ft_peak;

/* Create a plan on the current HIP device: validates the description, builds
 * the radix schedule of every transform length and uploads the FP64-derived
 * twiddle tables (the only allocation the library makes).
 * Returns FT_ERR_UNSUPPORTED_SIZE when a length has no compiled kernel. */
ft_status funnel_plan_create(const ft_plan_desc* desc, ft_plan** out);

/* One image of a ragged batch.  Images of different sizes go in one call;
 * each image's planes (regular then inverse, Np = rows+cols) start at
 * plane_offset.  Offsets are in floats from the images / planes base and must
 * be multiples of 4 (16-byte alignment).  The caller keeps the regions
 * disjoint; the library cannot see the buffers' extent.
 * Unlike a uniform plan's description, an image has no padded_len (ragged
 * images always use Np = rows+cols, Sec. 4.2) and a ragged plan has no
 * precision or NVMT flag: ragged batches run the FP32 path with the linear
 * NVMT. */
typedef struct {
  int32_t rows;          /* N, even, >= 4 */
  int32_t cols;          /* M, even, >= 4 */
  int64_t image_offset;  /* floats from the images base */
  int64_t plane_offset;  /* floats from the planes base */
} ft_image_desc;

/* Create a plan for a ragged batch: images are grouped into size classes,
 * each with its own radix schedule, tile variants, twiddles and workspace
 * region.  The classes of a call run concurrently on streams the plan owns,
 * forked from and joined back to the caller's stream with events (the call
 * is still stream-ordered and can be captured into a graph).  A ragged plan
 * must not be used from two host threads at once. */
ft_status funnel_plan_create_ragged(const ft_image_desc* images, int32_t count, int32_t spaces, ft_plan** out);

/* Schedules of a ragged plan's launches.
 *   FT_SCHEDULE_CLASS_STREAMS (the default): each size class runs its own
 *     three launches per direction on a stream of the plan's, concurrently
 *     with the other classes (forked from and joined back to the caller's
 *     stream), with the tile variants of each class and launch.
 *   FT_SCHEDULE_QUEUE: one persistent launch per pass kind for the whole
 *     batch -- forward A, B, C; adjoint C^T, B^T and A^T (inverse space, then
 *     regular space) -- whose blocks take (class, space, image, tile) items
 *     from a device-side work queue, longest transforms first, until it is
 *     empty.  Each length has a fixed tile shape there (16 or 32 elements per
 *     thread for the column passes, per launch); the queue counters live in
 *     the workspace.  Available when every class's lengths have queue
 *     kernels: Np in {560, 1120, 2000, 3000} and row lengths in {240, 320,
 *     480, 640, 720, 1080, 1280, 1920} (the camera formats 240x320, 480x640,
 *     720x1280 and 1080x1920), FP32, linear NVMT, at most 16 class x space
 *     segments; else FT_ERR_UNSUPPORTED_SIZE.
 * funnel_autotune times both schedules of a ragged plan and keeps the faster.
 * Both give the same results (bitwise, when the classes' tile variants have
 * 16 elements per thread and the queue's column launches shape 0). */
enum { FT_SCHEDULE_CLASS_STREAMS = 0, FT_SCHEDULE_QUEUE = 1 };
ft_status funnel_plan_set_schedule(ft_plan* plan, int32_t schedule);
ft_status funnel_plan_schedule(const ft_plan* plan, int32_t* schedule);

/* Release the plan's tables.  NULL is accepted. */
void funnel_plan_destroy(ft_plan* plan);

/* Bytes of device workspace funnel_forward and funnel_adjoint need. */
ft_status funnel_workspace_size(const ft_plan* plan, size_t* bytes);

/* Floats of parameter plane per image (regular Np*M and/or inverse Np*N);
 * for a ragged plan, the extent of the whole planes buffer. */
ft_status funnel_plane_elems(const ft_plan* plan, size_t* floats_per_image);

/* Floats the images and the planes buffers of a call must span. */
ft_status funnel_buffer_elems(const ft_plan* plan, size_t* image_floats, size_t* plane_floats);

/* Number of size classes (1 for a uniform batch). */
ft_status funnel_plan_classes(const ft_plan* plan, int32_t* n);

/* Padded length Np the plan uses (uniform plans only). */
ft_status funnel_padded_len(const ft_plan* plan, int32_t* np);

/* Forward funnel transform of a batch (Sec. 3.1 on the expanded image of
 * Sec. 4.2, for the spaces of the plan).
 *   images : device, float32 [batch][N][M]
 *   planes : device, float32 [batch][funnel_plane_elems], overwritten with P
 *            (signed; the brightness is |P|)
 *   ws     : device workspace of at least funnel_workspace_size bytes
 *   stream : hipStream_t (NULL = default stream) */
ft_status funnel_forward(const ft_plan* plan, const float* images, float* planes,
                         void* ws, size_t ws_bytes, void* stream);

/* Adjoint (transpose) of funnel_forward under the real inner products of
 * images and planes: d_images = F^T d_planes, the two spaces' contributions
 * summed.  d_images is overwritten.  Same layouts as funnel_forward.
 * Implemented as the transposed passes: (2/Np) DFT along y, conjugate DFT
 * along x' followed by the transposed interpolation (a gather with at most
 * two taps, no atomics), and the real part of the conjugate y DFT cropped to
 * the image rows. */
ft_status funnel_adjoint(const ft_plan* plan, const float* d_planes, float* d_images,
                         void* ws, size_t ws_bytes, void* stream);

/* ---- graphs ----
 * Capture the launches of funnel_forward and/or funnel_adjoint with fixed
 * buffers into an executable HIP graph, built once and replayed with one
 * call.  The graph reads and writes the buffers given here on every launch.
 * Building a graph synchronises nothing and allocates only the graph. */
enum { FT_GRAPH_FORWARD = 1u, FT_GRAPH_ADJOINT = 2u };
typedef struct ft_graph ft_graph;
ft_status funnel_graph_create(const ft_plan* plan, uint32_t what, const float* images, float* planes,
                              const float* d_planes, float* d_images, void* ws, size_t ws_bytes, ft_graph** out);
ft_status funnel_graph_launch(const ft_graph* graph, void* stream);
void funnel_graph_destroy(ft_graph* graph);

/* Bytes of device workspace funnel_peaks needs for a given K. */
ft_status funnel_peaks_workspace_size(const ft_plan* plan, int32_t K, size_t* bytes);

/* List-based peak detection of Sec. 4.4 on |P| of every plane: the first K
 * cells, in the order (|P| descending, linear index ascending), that precede
 * every other cell of their (2*radius+1)^2 neighbourhood, have |P| >= threshold
 * and are not border cells of the expansion (rows within 2 of y = +-N/2 at
 * slope bins -1..1; for the inverse plane N -> M) unless
 * FT_PEAK_KEEP_PAD_BOUNDARY is set.  This equals the visiting-list procedure
 * of the paper exactly.
 *   planes  : device, as written by funnel_forward
 *   K       : 1 .. 256
 *   radius  : 1 .. 8
 *   peaks   : device, ft_peak [batch][n_spaces][K], entries beyond the count
 *             are left unspecified
 *   n_found : device, int32 [batch][n_spaces]
 *   ws      : device scratch of funnel_peaks_workspace_size bytes: partial
 *             lists and one cutoff key per plane, all written by the call
 *             itself (no initialisation needed)
 * Spaces are ordered regular then inverse, as in the plane layout.  The
 * lists are the same on every run. */
ft_status funnel_peaks(const ft_plan* plan, const float* planes, int32_t K, float threshold,
                       int32_t radius, uint32_t flags, ft_peak* peaks, int32_t* n_found,
                       void* ws, size_t ws_bytes, void* stream);

/* Largest peak scratch funnel_peaks_noalloc can use (64 MiB per GPU). */
#define FT_PEAKS_SCRATCH_BYTES ((size_t)64 << 20)

/* funnel_peaks for callers that cannot allocate or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same lists, with the partial lists and per-plane cutoffs
 * in a static device array of FT_PEAKS_SCRATCH_BYTES that each GPU holds
 * from the first plan created on it until the process ends.  It calls no
 * allocator.  Arguments, checks and outputs as funnel_peaks; a plan and K
 * whose funnel_peaks_workspace_size exceeds FT_PEAKS_SCRATCH_BYTES give
 * FT_ERR_WORKSPACE_TOO_SMALL (use funnel_peaks with a workspace then; the
 * 32 x 1024^2 batch, both spaces, needs 17 MB at K = 16).  Every call on a
 * GPU shares that GPU's scratch, which keeps the last call's contents; each
 * call re-initialises what it reads (the cutoffs) by a fill kernel of its
 * own, so calls ordered one after the other (on one stream, or synchronised)
 * are fine, while calls that can run at the same time on one GPU
 * (unsynchronised streams, or host threads) race and give wrong lists. */
ft_status funnel_peaks_noalloc(const ft_plan* plan, const float* planes, int32_t K, float threshold,
                               int32_t radius, uint32_t flags, ft_peak* peaks, int32_t* n_found, void* stream);

/* One checked candidate line (Sec. 4.5). */
typedef struct {
  float profile[7];   /* mean image value on the line shifted by d = -D..D across it
                         (entries 2D+1 .. 6 are 0) */
  float contrast;     /* max(|profile[D] - (profile[0] + profile[2D]) / 2|,
                             |profile[2D] - profile[0]|): ridge or step edge */
  int32_t length;     /* line positions read (columns, regular; rows, inverse) */
  int32_t verified;   /* 1: length >= min_length and contrast >= min_contrast */
} ft_line_check;

/* Line verification of Sec. 4.5, steps 1-4, for every peak of a list written
 * by funnel_peaks: a band of 2*half_width+1 pixels centred on the peak's
 * candidate line (its slope and intercept; the record's space says whether
 * the line is row = slope*col + intercept or col = slope*row + intercept) is
 * integrated along the line and the band profile decides.  At each position
 * along the line (every column, regular; every row, inverse) the line crosses
 * at y = slope*pos + intercept, evaluated with one rounding; the samples
 * y + d, d = -D..D, are linear interpolations between the two pixels across
 * the line, and the position counts when all pixels floor(y)-D .. floor(y)+D+1
 * are inside the image.  A wrapping peak (Fig. 9) names a line that is not
 * in the image, so its flat band rejects it; the same line's peak in the
 * other space verifies.
 *   images     : device, the images the planes were computed from
 *   peaks, n_found : device, as written by funnel_peaks with the same K
 *   half_width : D in 1 .. 3 (a 3 .. 7 pixel band)
 *   min_contrast, min_length : the decision (min_contrast not NaN, min_length >= 0)
 *   out        : device, ft_line_check [batch][n_spaces][K]; slots beyond a
 *                plane's count are zero (verified = 0)
 * Enqueued on `stream`; no allocation, no synchronisation. */
ft_status funnel_verify(const ft_plan* plan, const float* images, const ft_peak* peaks, const int32_t* n_found,
                        int32_t K, int32_t half_width, float min_contrast, int32_t min_length, ft_line_check* out,
                        void* stream);

/* One refined peak. */
typedef struct {
  float col, row;     /* real-valued plane column and row of the local maximum */
  float value;        /* |P| there */
  float slope;        /* Eqs. 22-25 at the refined cell, in the form of the  */
  float intercept;    /* peak's ft_peak record (regular or inverse space)    */
  float shift;        /* distance from the detected cell, in cells (<= 1.42) */
} ft_refined;

/* Workspace of funnel_refine for lists of K peaks per plane (>= the
 * transform's workspace). */
ft_status funnel_refine_workspace_size(const ft_plan* plan, int32_t K, size_t* bytes);

/* Sub-cell refinement of the peaks of a funnel_peaks list.  Between cells
 * the plane is the last two steps of Sec. 3.1 with the x' DFT evaluated at a
 * real slope bin m (the DTFT of each NVMT-resampled row) and the inverse y
 * DFT at a real intercept y; it equals the plane at every cell.  From each
 * detected cell, `iters` safeguarded Newton steps climb |P| (the Newton step
 * when the Hessian is negative definite, else a gradient step of 1/4 cell;
 * steps clamped to 1/2 cell per axis and 1 cell in total), and Eqs. 22-25
 * read the line at the maximum: Eq. 19 focuses a line at real-valued
 * (m, y), so the refined parameters are closer to the line than the cell's.
 * Recomputes the forward spectra of `images` in the workspace (passes A and
 * B of funnel_forward), so it needs no planes.
 *   images        : device, the images the peaks were detected in
 *   peaks, n_found: device, as written by funnel_peaks with the same K
 *   iters         : 0 .. 16 (0: the records describe the cells themselves)
 *   out           : device, ft_refined [batch][n_spaces][K]; slots past a
 *                   plane's count are zero
 * Uniform plans only, row lengths (M, and N for the inverse space) powers of
 * two in 64 .. 4096, else FT_ERR_UNSUPPORTED_SIZE. */
ft_status funnel_refine(const ft_plan* plan, const float* images, const ft_peak* peaks, const int32_t* n_found,
                        int32_t K, int32_t iters, ft_refined* out, void* ws, size_t ws_bytes, void* stream);

/* ---- kernel timing (for measurement tools) ----
 * When enabled on a plan, every funnel_forward / funnel_adjoint call records a
 * HIP event pair around each kernel it launches, on the call's stream, and
 * notes that kernel's algorithmic HBM bytes (each input read once, each
 * output written once).  Enabling allocates the events (up to max_records
 * launches are kept; later launches are not recorded).  A plan being profiled
 * must not be used from two host threads at once. */
typedef struct {
  char name[40];          /* pass name, e.g. "regular.A" */
  int32_t launches;       /* launches recorded */
  float total_ms;         /* summed event time */
  double bytes_per_launch;/* algorithmic bytes moved by one launch */
} ft_kernel_time;

ft_status funnel_profile_enable(ft_plan* plan, int32_t max_records);
/* Synchronises on the recorded events, aggregates them per kernel name into
 * out[0 .. *n-1] (at most cap entries) and clears the records. */
ft_status funnel_profile_read(ft_plan* plan, ft_kernel_time* out, int32_t cap, int32_t* n);
ft_status funnel_profile_disable(ft_plan* plan);

/* ---- tile variants and autotuning ----
 * Every pass kernel exists in several tile shapes (elements per thread,
 * columns or rows per block).  A plan starts from a default per launch;
 * funnel_autotune tries every shape of every launch on the plan's real sizes,
 * one launch after the other in two sweeps, scoring each by the time of its size class's
 * whole forward + adjoint chain (allocating and freeing its own scratch
 * buffers and synchronising the stream), and keeps the best.  The reported
 * times (ft_tune_result.ms, ms_default) are those chain times.  Launches ("roles") are numbered
 *   0..5  forward  regular A, B, C, inverse A, B, C
 *   6..11 adjoint  regular Ct, Bt, At, inverse Ct, Bt, At
 * For a ragged plan, class c's launches are roles 12*c .. 12*c+11; a ragged
 * plan whose lengths have queue kernels then also times its two schedules
 * (FT_SCHEDULE_*, with each queue column launch's tile shape) and keeps the
 * faster, reported as a last result named "schedule" (variant = the
 * schedule, ms_default = the class-streams time).
 * A plan being tuned must not be used concurrently. */
typedef struct {
  char name[40];       /* role name, e.g. "fwd.regular.C" */
  int32_t variant;     /* chosen tile variant */
  int32_t n_tried;     /* variants timed */
  float ms;            /* best chain time with the chosen variant */
  float ms_default;    /* chain time with the variant the plan had before */
} ft_tune_result;

ft_status funnel_autotune(ft_plan* plan, void* stream, ft_tune_result* out, int32_t cap, int32_t* n);
/* Current variant of each role, 12 per size class (-1 for roles the plan does not run). */
ft_status funnel_plan_variants(const ft_plan* plan, int32_t* variants, int32_t cap);
/* Force one role's variant; FT_ERR_INVALID_ARG if that shape has no kernel. */
ft_status funnel_plan_set_variant(ft_plan* plan, int32_t role, int32_t variant);

/* ---- volumes (App. A) ----
 * The funnel transform of a volume V[z][y][x] maps planes to points: the
 * same steps with one more axis,
 *
 *   S(x, y, w3)   = DFT_z of the expanded volume            (Eq. A.2)
 *   g(x', y', w3) = S(x'/s, y'/s, w3), s = w3/w_max         (Eq. A.3; bilinear
 *                                                            interpolation)
 *   G(w1, w2, w3) = 2D DFT over x', y'                      (Eq. A.4)
 *   P(w1, w2, z)  = inverse DFT_w3 of G                     (Eqs. A.5, A.9)
 *
 * Conventions (as for images, per axis; stated for the z space):
 *   - volume V[s][r][c]: Nz slices (depth, z), Ny rows (y), Nx columns (x),
 *     row-major float32, all even and >= 4; volumes of a batch are
 *     contiguous (stride Nz*Ny*Nx).
 *   - the z axis is expanded to Lp = Nz + Ny + Nx (or padded_len) with
 *     (Lp-Nz)/2 zero slices in front: a plane with |a|, |b| <= 1 moves by at
 *     most (Nx+Ny)/2 slices over the volume.  Centred z, y, x.
 *   - w_max = pi, s = 2 n3 / Lp for n3 = 1 .. Lp/2-1; DC and Nyquist zero.
 *   - bilinear NVMT: linear interpolation along x and along y, each as the
 *     image NVMT (exact integer floors of (x' Lp + Nx n3)/(2 n3) and of
 *     (y' Lp + Ny n3)/(2 n3)), the weights multiplied.
 *   - parameter spaces.  Eq. A.9 focuses the planes whose depth changes by at
 *     most one slice per row and column (|a|, |b| <= 1).  Steeper planes are
 *     found by the same transform with x or y as the depth axis, the 3D
 *     counterpart of the image's inverse space.  Each space runs on the
 *     volume with its axes in the order (depth, rows, cols):
 *       FT_VOL_SPACE_Z: (z, y, x), the volume as stored;
 *       FT_VOL_SPACE_X: (x, z, y);
 *       FT_VOL_SPACE_Y: (y, z, x).
 *     Every space expands its depth axis to the same Lp = Nz + Ny + Nx (or
 *     padded_len).
 *   - parameter volume of a space: float32 P[Lp][rows][cols], slice =
 *     z + Lp/2, row = m2 + rows/2, column = m1 + cols/2.  A plane
 *     depth = a*col + b*row + c (the space's voxel indices, |a|, |b| <= 1)
 *     focuses at m1 = -a cols/2, m2 = -b rows/2, z = c + a cols/2 +
 *     b rows/2 - depth/2.  A volume's parameter volumes are contiguous in
 *     the order z, x, y (the spaces the plan computes), and volumes follow
 *     each other with the stride of funnel_volume_param_elems().
 * Sizes with kernels: Lp a compiled column length (as Np for images); for
 * each space computed, its cols a compiled row length (as M) and its rows in
 * {32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512, 640, 768, 1024}; each
 * parameter volume below 2 GiB.  FP32.  Ownership, threading and errors as
 * for image plans. */
enum { FT_VOL_SPACE_Z = 1, FT_VOL_SPACE_X = 2, FT_VOL_SPACE_Y = 4, FT_VOL_SPACE_ALL = 7 };
typedef struct ft_volume_plan ft_volume_plan;

typedef struct {
  int32_t batch;       /* number of volumes, >= 1 */
  int32_t depth;       /* Nz, slices */
  int32_t rows;        /* Ny */
  int32_t cols;        /* Nx */
  int32_t padded_len;  /* Lp; 0 means Nz+Ny+Nx; else even and >= Nz+Ny+Nx */
  int32_t spaces;      /* a non-empty set of FT_VOL_SPACE_Z / _X / _Y */
  uint32_t flags;      /* 0 */
} ft_volume_desc;

ft_status funnel_volume_plan_create(const ft_volume_desc* desc, ft_volume_plan** out);
void funnel_volume_plan_destroy(ft_volume_plan* plan);
ft_status funnel_volume_padded_len(const ft_volume_plan* plan, int32_t* nzp);
/* Floats of one volume's parameter volumes (all spaces of the plan). */
ft_status funnel_volume_param_elems(const ft_volume_plan* plan, size_t* floats_per_volume);
/* Bytes of device workspace funnel_volume_forward needs: the largest space's
 * half spectrum, (Lp/2-1) * rows * cols complex values per volume, and for
 * the y space a slice-transposed copy of the volumes. */
ft_status funnel_volume_workspace_size(const ft_volume_plan* plan, size_t* bytes);

/* Forward transform of a batch of volumes (App. A, Eqs. A.2-A.5), in every
 * space of the plan.
 *   volumes : device, float32 [batch][Nz][Ny][Nx]
 *   params  : device, float32 [batch][funnel_volume_param_elems], overwritten
 *   ws      : device workspace of at least funnel_volume_workspace_size bytes
 * Per space four launches: DFT along the depth axis, NVMT + DFT along x',
 * NVMT + DFT along y' (bilinear interpolation is the product of the two
 * linear ones), inverse DFT along w3 with 1/Lp; the y space first transposes
 * every slice so that its depth lines are contiguous. */
ft_status funnel_volume_forward(const ft_volume_plan* plan, const float* volumes, float* params, void* ws,
                                size_t ws_bytes, void* stream);

/* One detected 3D peak and its plane (Eq. A.9 read backwards). */
typedef struct {
  int32_t volume;
  int32_t space;       /* 0: z space, 1: x space, 2: y space */
  int32_t z;           /* parameter-volume slice (intercept bin) */
  int32_t row;         /* m2 + rows/2 */
  int32_t col;         /* m1 + cols/2 */
  float value;         /* |P| */
  float a, b, c;       /* the plane depth = a*col + b*row + c in the space's
                          voxel indices: z space slice = a*x + b*y + c,
                          x space x = a*y + b*z + c, y space y = a*x + b*z + c */
} ft_plane_peak;

ft_status funnel_volume_peaks_workspace_size(const ft_volume_plan* plan, int32_t K, size_t* bytes);
/* The list rule of Sec. 4.4 in three dimensions: the first K cells, in the
 * order (|P| descending, linear index ascending), that precede every other
 * cell of their (2*radius+1)^3 neighbourhood (toroidal, or clamped with
 * FT_PEAK_CLAMP_BORDER), have |P| >= threshold and are not cells where the
 * expansion's faces focus (slices within 2 of z = -+Nz/2 at m1, m2 in
 * {-1, 0, 1}) unless FT_PEAK_KEEP_PAD_BOUNDARY is set.
 *   K       : 1 .. 256;  radius : 1 or 2
 *   peaks   : device, ft_plane_peak [batch][n_spaces][K] (entries beyond the
 *             count unspecified), spaces in the order z, x, y
 *   n_found : device, int32 [batch][n_spaces]
 *   ws      : device scratch of funnel_volume_peaks_workspace_size bytes
 *             (partial lists and one cutoff key per volume, written by the
 *             call itself)
 * The lists are the same on every run. */
ft_status funnel_volume_peaks(const ft_volume_plan* plan, const float* params, int32_t K, float threshold,
                              int32_t radius, uint32_t flags, ft_plane_peak* peaks, int32_t* n_found, void* ws,
                              size_t ws_bytes, void* stream);

/* Tile variants of the four launches of each space (role 4*s + r, s = 0 z,
 * 1 x, 2 y space; r = 0 depth DFT, 1 x' pass, 2 y' pass, 3 inverse w3 DFT;
 * -1 for a space the plan does not compute), autotuning over the whole
 * forward chain, and kernel timing, as for image plans. */
ft_status funnel_volume_variants(const ft_volume_plan* plan, int32_t* variants, int32_t cap);
ft_status funnel_volume_set_variant(ft_volume_plan* plan, int32_t role, int32_t variant);
ft_status funnel_volume_autotune(ft_volume_plan* plan, void* stream, ft_tune_result* out, int32_t cap, int32_t* n);
ft_status funnel_volume_profile_enable(ft_volume_plan* plan, int32_t max_records);
ft_status funnel_volume_profile_read(ft_volume_plan* plan, ft_kernel_time* out, int32_t cap, int32_t* n);
ft_status funnel_volume_profile_disable(ft_volume_plan* plan);

/* Human-readable name of a status. */
const char* funnel_status_string(ft_status status);

/* Message of the last failed call on this thread ("" if none). */
const char* funnel_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FUNNEL_H */
