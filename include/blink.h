/*
 * blink.h - C ABI of the MI355X (gfx950) dirty-imaging library libblink.so.
 *
 * For every (timestep, channel) image the library grids the visibilities of
 * all baselines onto an N x N uv grid and applies the 2D inverse FFT; the real
 * part, shifted so that the phase centre sits at the image centre, is the
 * dirty image (Sokolowski et al., "High-Time Resolution GPU Imager for FRB
 * searches at low radio frequencies": Sec. 4.3 Eqs. 4-6, Sec. 4.4 Eqs. 7-9,
 * Sec. 5.2.1-5.2.2, Sec. 5.2.4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - blink_problem and blink_inputs are host structs, read during the call
 *   only. Every array they (or the calls) point to is DEVICE memory, owned by
 *   the caller; the library never allocates device memory, frees or
 *   synchronises (the one exception, blink_image_batch_timed, is an
 *   instrumentation call that waits for its own timing events).
 * - Scratch memory comes from a caller-provided device workspace of at least
 *   blink_workspace_size() bytes, 256-byte aligned. Its contents on entry are
 *   irrelevant; it must not be shared by calls that may run concurrently.
 * - Work is enqueued on the caller's HIP stream `stream`. Nothing inside a
 *   call blocks the host, so calls may be captured into a HIP graph.
 * - Arrays are C-contiguous, row-major. blink_c32 is {float re, im}, the
 *   layout of torch.complex64 / std::complex<float>.
 * - Argument errors are detected on the host before anything is enqueued and
 *   leave every output untouched. A failed kernel launch returns BLINK_E_HIP.
 *   Faults during execution surface at the caller's next synchronisation.
 * - No mutable global state, so calls are thread-safe; the one exception is
 *   blink_image_batch_noalloc, whose per-GPU scratch array is shared by all
 *   of its calls on that GPU (see there).
 *
 * Geometry and the readings of the paper used throughout
 * ------------------------------------------------------
 * - uvw_m[t][b] = (u, v, w) of baseline b at timestep t in metres; w enters
 *   only the phase rotation and the re-projection below (otherwise the array
 *   is imaged as coplanar, phased to zenith, Sec. 4.3 Eq. 5).
 * - Cells per metre of channel c: s_c = (freq_hz[c] * (N * pixscale)) / c0 with
 *   c0 = 299792458 m/s, evaluated in IEEE double in that order (Eq. 9 gives
 *   the cell du = 1/(N dx) wavelengths; Sec. 5.2.4 computes the channel
 *   frequency and wavelength in double). freq_hz must be finite and > 0
 *   (device memory, so not checked): other values give unspecified images,
 *   but every memory access stays within the arrays.
 * - Cell of baseline b: i_u = rint(u * s_c), i_v = rint(v * s_c) (one double
 *   product, round half to even). The baseline is kept iff it is not flagged,
 *   u and v are finite, |i_u| < N/2 and |i_v| < N/2; kept baselines are
 *   counted at (i_v mod N, i_u mod N) with value V' and at the mirror cell
 *   with conj(V') (the input holds each antenna pair once).
 * - V' = gains[ant1[b]] * conj(gains[ant2[b]]) * V when gains are given
 *   (post-correlation calibration, Sec. 4.2 (ii)); for FP16/BF16 storage
 *   V = (float(q_re) + i float(q_im)) * vis_scale[c].
 * - Weighting (Sec. 4.4.2): NATURAL cell value = sum, W = sum of counts;
 *   UNIFORM cell value = sum / count, W = number of occupied cells.
 * - Image: unnormalised inverse transform exp(+2 pi i (k.q)/N), real part,
 *   FFT shift (Sec. 5.2.2), times 1/W when norm = BLINK_NORM_WEIGHTS (W = 0
 *   gives zeros), then the central M x M cutout. Layout [m][l]: row follows
 *   v (m), column follows u (l), phase centre at [M/2][M/2].
 * - Gridding kernel (kernel_support = W >= 1; the anti-aliasing convolution
 *   that Sec. 4.4.1 describes and the paper's imager leaves out): a baseline
 *   at the exact cell position x = (u s_c, v s_c) adds
 *   C(i - x_u) C(j - x_v) V' to every cell with |i - x_u| <= W/2 and
 *   |j - x_v| <= W/2 (and the same weight times conj(V') at the mirror
 *   cells), C(d) = I0(beta sqrt(1 - (2d/W)^2)) / I0(beta). It is kept iff
 *   that whole footprint satisfies |i| < N/2, |j| < N/2. W = the sum of all
 *   weights added. UNIFORM (Sec. 4.4.2 read together with 4.4.1) multiplies
 *   every weight of baseline b by 1 / n_b, n_b the number of kept entries,
 *   direct and mirrored, whose nearest cell (rint(x_u), rint(x_v)) is b's
 *   own (so the one-cell box kernel, W = 1 with beta = 0, gives the
 *   nearest-cell uniform image). Each image pixel at offset
 *   (q_m, q_l) from the centre is divided by c(q_l/N) c(q_m/N), c the
 *   kernel's continuous Fourier transform normalised to c(0) = 1:
 *   c(xi) = [sinh(z)/z] / [sinh(beta)/beta], z = sqrt(beta^2 - (pi W xi)^2)
 *   (sin(|z|)/|z| where pi W |xi| > beta). Weights are evaluated in FP32 from
 *   the FP64 distances, by a polynomial within 2e-8 of C (plus FP32 rounding)
 *   up to beta of about 70, else by the FP32 Bessel routine; blink_grid
 *   returns counts of contributions per cell. blink_degrid_adjoint degrids
 *   with the same kernel (see there).
 * - Phase rotation (phase_l, phase_m != 0; Sec. 4.2 (iii)): correlation
 *   phases the visibilities to zenith; each V' is multiplied by
 *   exp(+2 pi i (u l0 + v m0 + w (n0 - 1)) nu_c / c0), n0 = sqrt(1 - l0^2 -
 *   m0^2), so that a source at (l0, m0) becomes a constant and images at the
 *   centre. With reproject = 0, (u, v, w) are not re-projected: the image
 *   stays on the zenith tangent plane, shifted by (l0, m0). With reproject =
 *   1 the image lies on the tangent plane at s0 = (l0, m0, n0): each baseline
 *   is gridded at u' = b.e_u', v' = b.e_v' (metres, in double), the axes
 *   e_u' = (n0 + m0^2 k, -l0 m0 k, -l0), e_v' = (-l0 m0 k, n0 + l0^2 k, -m0),
 *   k = 1 / (1 + n0): the zenith frame's east and north axes carried by the
 *   smallest rotation that takes zenith to s0; a source at direction
 *   cosines (l', m') of that frame images at (l', m'). reproject is ignored
 *   at (0, 0) and must be 0 or 1. The delay is formed in double at the
 *   sort, the phase in cycles in double, its sine and cosine in float.
 *   blink_degrid_adjoint applies the conjugate factor to the gradients.
 * - Cable correction (blink_inputs.cable_m != NULL; Sec. 4.2 (i)): antenna
 *   a's signal path is longer by the electrical length l_a metres, which
 *   multiplies its voltage by exp(-2 pi i nu l_a / c0); each V' of baseline
 *   (ant1, ant2) is multiplied by exp(+2 pi i (l_ant1 - l_ant2) nu_c / c0).
 *   The term adds to the geometric delay above (one factor per visibility).
 *   It needs ant1, ant2 and n_ant >= 1; an antenna index outside
 *   [0, n_ant) contributes no cable term (and, with gains, a zero gain).
 *   blink_degrid_adjoint applies the conjugate factor to the gradients.
 *   Per-antenna complex gains (Sec. 4.2 (ii)) are the `gains` input.
 */
#ifndef BLINK_H
#define BLINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* blink_stream_t;   /* the same handle as hipStream_t */

typedef struct { float re, im; } blink_c32;

typedef enum {
  BLINK_OK = 0,
  BLINK_E_ARG = -1,          /* null required pointer, bad enum or tunable, non-finite or <= 0 pixscale */
  BLINK_E_SIZE = -2,         /* negative sizes, odd N or M, M > N, element count overflow   */
  BLINK_E_UNSUPPORTED = -3,  /* N without a compiled transform plan, a combination not built,
                                or a tile width whose workgroup does not fit in LDS            */
  BLINK_E_WORKSPACE = -4,    /* workspace null, misaligned or smaller than required          */
  BLINK_E_HIP = -5           /* a HIP launch failed (hipGetLastError after the enqueue)       */
} blink_status;

typedef enum { BLINK_NATURAL = 0, BLINK_UNIFORM = 1 } blink_weighting;
typedef enum { BLINK_VIS_C64 = 0, BLINK_VIS_F16 = 1, BLINK_VIS_BF16 = 2 } blink_vis_type;
typedef enum { BLINK_NORM_NONE = 0, BLINK_NORM_WEIGHTS = 1 } blink_norm;
typedef enum {
  BLINK_CALL_GRID = 0,       /* blink_grid            */
  BLINK_CALL_IMAGE = 1,      /* blink_image_batch     */
  BLINK_CALL_ADJOINT = 2     /* blink_degrid_adjoint  */
} blink_call;

typedef struct {
  int32_t n_time;        /* T: timesteps in the cube                                  */
  int32_t n_chan;        /* C: channels                                               */
  int32_t n_bl;          /* B: baselines (each antenna pair once)                     */
  int32_t n_ant;         /* A: antennas (gains length; may be 0 without gains)        */
  int32_t grid_n;        /* N: even, one of the sizes reported by blink_supported_n   */
  int32_t out_n;         /* M: even, M <= N; central M x M cutout of the N x N image   */
  double  pixscale;      /* dx: pixel size in direction-cosine units (> 0, finite)     */
  int32_t weighting;     /* blink_weighting                                           */
  int32_t norm;          /* blink_norm                                                */
  int32_t vis_type;      /* blink_vis_type                                            */
  int32_t chunk_images;  /* images per internal chunk; 0 = library default            */
  int32_t cols_per_wg;   /* u-cell columns per workgroup of the image path's column    */
                         /* kernel: 0 = library default, else 2, 4 or 8                */
  int32_t rows_wg;       /* row pass: 0 = one workgroup per row tile, > 0 = that many  */
                         /* persistent workgroups walking the row tiles                */
  int32_t kernel_support;/* gridding kernel: 0 = nearest cell (the paper's imager);   */
                         /* 1..16 = separable Kaiser-Bessel of that support W in cells */
                         /* with the image-domain correction (see below)               */
  double  kernel_beta;   /* Kaiser-Bessel shape; < 0 = pi sqrt(0.5625 W^2 - 0.8)       */
                         /* (needs W >= 2); at most 80; ignored when kernel_support = 0 */
  double  phase_l;       /* phase centre (direction cosines relative to zenith) for    */
  double  phase_m;       /* the geometric rotation at load; (0, 0) = zenith, none;     */
                         /* l^2 + m^2 < 1                                               */
  int32_t reproject;     /* 1: image on the tangent plane at (phase_l, phase_m)        */
                         /* (baselines re-projected, see below); 0: zenith plane       */
} blink_problem;

typedef struct {          /* device pointers; the optional ones may be NULL            */
  const void*      vis;       /* [T][C][B] blink_c32, or [T][C][B][2] f16 / bf16 pairs  */
  const float*     vis_scale; /* [C] dequantisation scale; required for f16 / bf16      */
  const double*    uvw_m;     /* [T][B][3] metres                                       */
  const double*    freq_hz;   /* [C] Hz                                                  */
  const uint8_t*   flags;     /* [T][B] nonzero = flagged for every channel, or NULL    */
  const int32_t*   ant1;      /* [B] antenna of the first input (required with gains)    */
  const int32_t*   ant2;      /* [B] antenna of the second input                         */
  const blink_c32* gains;     /* [A] per-antenna complex gains, or NULL                  */
  const double*    cable_m;   /* [A] electrical cable length per antenna (m), or NULL    */
} blink_inputs;

/* Human-readable name of a status code (static string). */
const char* blink_status_string(blink_status s);

/* 1 if a transform plan for length n is compiled in, else 0. */
int32_t blink_supported_n(int32_t n);

/* Bytes of workspace that `call` needs for problem `p` (0 on invalid input). */
size_t blink_workspace_size(const blink_problem* p, int32_t call);

/*
 * blink_grid: the gridding step alone (Sec. 5.2.1 steps 1-3, Sec. 4.4.2).
 * Writes, for every image i = t*C + c:
 *   grid[i][k_v][k_u]  blink_c32, the WEIGHTED grid that the inverse FFT
 *                      consumes (natural: cell sums; uniform: sum / count),
 *                      DC at [0][0], both the cell and its mirror filled;
 *   counts[i][k_v][k_u] int32 visibilities per cell (NULL to skip);
 *   weight_sum[i]      float W (NULL to skip);
 *   n_dropped[i]       int32 unflagged baselines outside the grid or with
 *                      non-finite u, v (NULL to skip).
 * grid is [T*C][N][N]; out_n and norm are ignored.
 */
blink_status blink_grid(const blink_problem* p, const blink_inputs* in,
                        blink_c32* grid, int32_t* counts, float* weight_sum,
                        int32_t* n_dropped, void* workspace, size_t ws_bytes,
                        blink_stream_t stream);

/*
 * blink_fft2d: batched unnormalised 2D C2C transform of [batch][n][n]
 * complex arrays: out[q] = sum_k in[k] exp(sign * 2 pi i (k_v q_v + k_u q_u) / n)
 * (sign = +1 is the inverse transform of Sec. 5.2.2, -1 the forward one).
 * in == out is allowed; otherwise the buffers must not overlap. No workspace.
 */
blink_status blink_fft2d(const blink_c32* in, blink_c32* out, int32_t batch,
                         int32_t n, int32_t sign, blink_stream_t stream);

/*
 * blink_image_batch: the whole path, visibilities -> dirty images, for all
 * T*C images of the cube (Sec. 5.2.4 "layers"): images [T*C][M][M] float,
 * weight_sum [T*C] float W (NULL to skip). Ragged batches (different flag
 * counts per timestep) need no padding.
 */
blink_status blink_image_batch(const blink_problem* p, const blink_inputs* in,
                               float* images, float* weight_sum,
                               void* workspace, size_t ws_bytes,
                               blink_stream_t stream);

/*
 * blink_image_batch_noalloc: blink_image_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation). Same arguments without the
 * workspace, same results bit for bit. Its scratch memory is a fixed
 * array of BLINK_NOALLOC_SCRATCH_BYTES in the library's code object, one
 * copy per GPU, held until the process ends; the call itself allocates
 * nothing. The array of the CURRENT device is used (its address is looked
 * up once per device on the first call there), so `stream` must belong to
 * the current device. The cube is imaged in blocks of whole timesteps whose
 * workspace fits the array, with chunk_images as an upper bound on the
 * images per internal chunk. Returns BLINK_E_WORKSPACE when the workspace
 * of one timestep with a single-image chunk exceeds the array (e.g.
 * N = M = 4096, whose half spectrum alone is 64 MiB per image), BLINK_E_HIP
 * if the address lookup fails, and the errors of blink_image_batch
 * otherwise.
 * Every call on a GPU shares that GPU's array: calls that may overlap on one
 * GPU (other streams, other host threads) race and must be serialised by
 * the caller. Nothing in the array needs to be cleared between calls.
 */
#define BLINK_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
blink_status blink_image_batch_noalloc(const blink_problem* p, const blink_inputs* in,
                                       float* images, float* weight_sum,
                                       blink_stream_t stream);

/*
 * blink_degrid_adjoint: gradients of a real loss L through blink_image_batch,
 * given image_grad = dL/d(images) [T*C][M][M] float:
 *   vis_grad[t][c][b]  = dL/dRe V + i dL/dIm V   (blink_c32, all baselines;
 *                        zero for flagged or dropped ones; with FP16/BF16
 *                        storage, the gradient with respect to the
 *                        dequantised V);
 *   gain_grad[a]       = dL/dRe g + i dL/dIm g   (NULL to skip; needs gains,
 *                        ant1, ant2).
 * weight_sum [T*C] float: the weight sums W that blink_image_batch returned
 * for the same problem and inputs, or NULL, in which case they are counted
 * again from the baseline lists (device memory, not checked: other values
 * scale the gradient of each image by their ratio to the true W).
 * The map V -> image is linear (W and the counts depend only on geometry and
 * flags), so this is the exact adjoint: zero-pad, 1/W, inverse shift, forward
 * transform, cell weight, gather at +k and -k (degridding), times the
 * conjugate of the rotation / cable factor when one is applied. With a
 * gridding kernel (kernel_support > 0) the image gradient is first divided by
 * the same correction c(q_l/N) c(q_m/N), and the degridding sums, for each
 * kept baseline, C(i - x_u) C(j - x_v) (times 1/n_b with UNIFORM) over its
 * footprint cells of the transformed gradient, plus the conjugate of the same
 * sum over its mirror cells; without weight_sum, W is counted again by the
 * forward column pass.
 */
blink_status blink_degrid_adjoint(const blink_problem* p, const blink_inputs* in,
                                  const float* image_grad, const float* weight_sum,
                                  blink_c32* vis_grad, blink_c32* gain_grad, void* workspace,
                                  size_t ws_bytes, blink_stream_t stream);

/*
 * Per-kernel timing of the image path (instrumentation for benchmarks and
 * profiling; not for graph capture). Kernel classes of blink_image_batch:
 *   0 = per-timestep sort (all its launches), 1 = cell bounds,
 *   2 = gridding + column inverse transform, 3 = row inverse transform with
 *   the fused shift / 1/W / cutout.
 */
#define BLINK_KCLASS_COUNT 4
typedef struct {
  double  ms[BLINK_KCLASS_COUNT];        /* summed kernel time, milliseconds   */
  int64_t launches[BLINK_KCLASS_COUNT];  /* number of launches of the class    */
} blink_kernel_times;

/*
 * Same work and results as blink_image_batch, with a HIP event recorded on
 * `stream` before and after every launch. Blocks the host until the last
 * event completes, then writes the per-class sums into *times (which must be
 * non-null). Results are bitwise identical to blink_image_batch.
 */
blink_status blink_image_batch_timed(const blink_problem* p, const blink_inputs* in,
                                     float* images, float* weight_sum, void* workspace,
                                     size_t ws_bytes, blink_stream_t stream,
                                     blink_kernel_times* times);

/*
 * blink_dynamic_spectra: per-pixel time series of an image cube, with a
 * reference image subtracted (Sec. 2: dynamic spectra of every pixel are
 * formed from the cube of images and searched for transients; dirty-image
 * artefacts are removed by subtracting a reference image of the same field,
 * which Sec. 4.3 takes as the preceding image, an average of the preceding
 * images or a model image).
 *   images  [n_time][n_chan][n_pix] float (n_pix = M*M, the images of
 *           blink_image_batch as they come out), device, read only;
 *   spectra [n_pix][n_chan][n_time] float, device, written; must not
 *           overlap images;
 *   ref_mode BLINK_REF_NONE:  spectra[p][c][t] = images[t][c][p];
 *            BLINK_REF_MEAN:  images[t][c][p] minus the mean of the
 *                             k = min(ref_len, t) preceding images at (c, p),
 *                             evaluated in double and rounded once; 0 at t = 0
 *                             (ref_len in 1..BLINK_REF_MAX_LEN; 1 = preceding
 *                             image);
 *            BLINK_REF_MODEL: images[t][c][p] - ref_image[c][p] (FP32);
 *   ref_image [n_chan][n_pix] float, device; required for BLINK_REF_MODEL,
 *           ignored otherwise.
 * Errors: BLINK_E_SIZE for negative sizes, n_chan > 65535 or element counts
 * beyond 2^62; BLINK_E_ARG for null required pointers, an unknown mode or
 * ref_len out of range. No workspace; enqueued on `stream`.
 */
typedef enum { BLINK_REF_NONE = 0, BLINK_REF_MEAN = 1, BLINK_REF_MODEL = 2 } blink_reference;

/*
 * blink_correlate: the X-engine of an FX correlator (Sec. 4.1): for every
 * integration t and channel c, the products of the channelised complex
 * voltages of all antenna pairs, accumulated over the integration's samples:
 *   V_ij = sum_s x_i(s) conj(x_j(s))   (the conjugate on the second antenna;
 *                                        the equation as printed omits it)
 *   volt  [n_time][n_chan][n_ant][n_samp][2] int8 (real, imaginary), device,
 *         16-byte aligned;
 *   vis   [n_time][n_chan][n_ant (n_ant - 1) / 2] blink_c32, device: pairs
 *         i < j in row-major upper-triangle order (the baseline order that
 *         blink_image_batch's inputs use with ant1 = i, ant2 = j);
 *   autos [n_time][n_chan][n_ant] float V_aa, device, or NULL.
 * Integer products on the matrix cores, summed exactly in int32, then
 * converted to float (exact below 2^24 in magnitude). The plain sum, not
 * the average, is returned.
 * Errors: BLINK_E_SIZE for negative sizes, n_ant < 2 with T*C > 0, n_samp not
 * a multiple of 16 or above 65520 (the int32 sums of 2 n_samp products of
 * magnitude up to 128^2 stay below 2^31), or counts beyond 2^62; BLINK_E_ARG for null
 * or misaligned required pointers. No workspace; enqueued on `stream`.
 */
blink_status blink_correlate(const int8_t* volt, int32_t n_time, int32_t n_chan, int32_t n_ant,
                             int32_t n_samp, blink_c32* vis, float* autos, blink_stream_t stream);
#define BLINK_REF_MAX_LEN 128
blink_status blink_dynamic_spectra(const float* images, int32_t n_time, int32_t n_chan, int32_t n_pix,
                                   int32_t ref_mode, int32_t ref_len, const float* ref_image,
                                   float* spectra, blink_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BLINK_H */
