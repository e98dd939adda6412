/*
 * recon.h — C ABI of the MI355X (gfx950) ordered-subset TV reconstruction library.
 *
 * Method: Ozaki et al., "Fast Statistical Iterative Reconstruction for MVCT in
 * TomoTherapy" (arXiv:1903.10088).  The library maximises the posterior of
 * section 2 (Eqs. 1-2: Poisson transmission likelihood plus a total-variation
 * prior, image constrained positive) by the gradient iteration of Eq. 3 with
 * the adaptive convergence parameter of Eqs. 4-5 (section 3.C.2), over
 * equal-interval view subsets with the prior weight scaled by the thinning
 * factor (section 3.D).  Every step runs in hand-written HIP kernels on the GPU.
 *
 * Conventions shared by all entry points
 *  - Units: lengths in mm, attenuation in 1/mm.  The step rule works in the
 *    paper's cm / (1/cm) internally; that conversion is hidden.
 *  - Image: float32, n*n, row-major, element [j][i] at j*n + i, pixel centre
 *    x = (i - (n-1)/2) * pixel_mm, y = (j - (n-1)/2) * pixel_mm.  The
 *    reconstruction disc is x^2 + y^2 <= (n * pixel_mm / 2)^2; outside it the
 *    iterate is held at zero.
 *  - Fan beam: view v has its source at SAD * (cos b, sin b),
 *    b = start_angle + arc v / n_views (counter-clockwise), arc = scan_arc_rad
 *    or 2 pi when that is 0; channel k lies on
 *    an arc centred on the source at fan angle g = (k - (n_channels-1)/2) * dg,
 *    dg = 2 * gamma_max / n_channels, gamma_max = fan_half_angle_rad or, when
 *    that is 0, asin(R / SAD) with R = n * pixel_mm / 2; the ray leaves the
 *    source towards angle b + pi + g.
 *  - Sinogram: float32 [view][channel], row-major.  "subset s" (0 <= s < M)
 *    means the views v with v mod M == s in increasing order; subset -1 means
 *    all views in natural order.
 *  - Device pointers: every float / double pointer marked d_ is device memory
 *    owned by the caller, contiguous, and must stay valid until the work
 *    queued on `stream` has finished.  `stream` is a hipStream_t (NULL = the
 *    null stream).  Calls are asynchronous unless stated otherwise.
 *  - Errors: every call returns a recon_status; nothing is thrown across the
 *    ABI.  recon_last_error() returns a message for the last failure on the
 *    calling thread.  A handle is not thread-safe; distinct handles may be used
 *    from distinct threads and streams.
 */
#ifndef RECON_H
#define RECON_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RECON_OK = 0,
    RECON_INVALID_ARG = 1, /* null pointer, bad size, unsupported geometry or parameter */
    RECON_DEVICE = 2,      /* a HIP runtime call failed */
    RECON_NUMERIC = 3,     /* a non-finite squared difference was met during an iteration */
    RECON_OOM = 4          /* device or host allocation failed */
} recon_status;

/* Fan-beam geometry.  Requirements: n >= 2, pixel_mm > 0, n_views >= 1,
 * 1 <= n_channels <= 65535, sad_mm > sqrt(2) * n * pixel_mm / 2 (the whole
 * pixel grid lies on the detector side of the source), full fan angle below
 * 90 degrees, 0 <= scan_arc_rad <= 2 pi.  sdd_mm is carried for completeness:
 * on an arc detector centred on the source it does not change any line
 * integral.  scan_arc_rad is the angular range the views sweep: 0 (or 2 pi)
 * is a full turn; a smaller value is limited-angle data (section 4,
 * reconstructed images: fewer projection data), its n_views views spaced
 * arc / n_views apart over [start, start + arc).  The iteration, projector and
 * backprojector take any arc; recon_fbp and recon_rebin_helical need a full
 * turn. */
typedef struct {
    int32_t n;
    int32_t reserved0;
    double pixel_mm;
    int32_t n_views;
    int32_t n_channels;
    double sad_mm;
    double sdd_mm;
    double fan_half_angle_rad;
    double start_angle_rad;
    double scan_arc_rad;
} recon_geometry;

/* Step rule and prior parameters (section 3.C).  Defaults (recon_default_params):
 * lambda0 0.01, lambda_inc 1e-4 (Eq. 4), lambda_dec 2e-4 (Eq. 5), lambda_min 1e-4
 * (floor; not in the paper), mu0_per_mm 0.005 (0.05/cm, section 3.C.2),
 * tv_eps_per_mm 1e-5 (smoothing of the TV norm; not in the paper),
 * lambda_compare 0, keep_best 0.
 * lambda_compare: 0 = Eqs. 4-5 compare f_n with the previous sub-iteration's
 *   f (the literal reading); 1 = with the f of the same subset one epoch (M
 *   sub-iterations) earlier, from the second epoch on (the first epoch
 *   compares with the previous sub-iteration).  Both readings take a tie as
 *   "not decreased".
 * keep_best: 1 = also keep the iterate at the minimum of the oscillating
 *   squared difference (section 4.B), taken per epoch: f summed over the
 *   sub-iterations n = eM .. eM + M - 1 (n counted from the fresh start); when
 *   an epoch's sum is below every earlier epoch's, the image that epoch ends
 *   with, mu^((e+1)M), is written to the caller's best-image buffer
 *   (recon_os_iterate_ex).  Not available to the batched entry points. */
typedef struct {
    double lambda0;
    double lambda_inc;
    double lambda_dec;
    double lambda_min;
    double mu0_per_mm;
    double tv_eps_per_mm;
    int32_t lambda_compare;
    int32_t keep_best;
} recon_params;

/* Resumable iteration state (host memory).  A zero-filled struct with
 * n_done = 0 starts a fresh run (best_f, epoch_sum and best_n are then
 * ignored and start at +infinity, 0 and 0). */
typedef struct {
    int32_t n_done;   /* sub-iterations completed so far */
    int32_t flags;    /* bit 0: a non-finite squared difference was met */
    double lambda;    /* convergence parameter of the last sub-iteration */
    double f_prev;    /* squared difference of the last sub-iteration */
    double best_f;    /* least epoch sum of f so far (+infinity before the first epoch ends) */
    double epoch_sum; /* sum of f over the current, unfinished epoch */
    int32_t best_n;   /* sub-iterations that produced the kept iterate (0: no epoch ended yet) */
    int32_t reserved;
} recon_state;

typedef struct recon_handle recon_handle;

void recon_default_params(recon_params* out);
const char* recon_status_string(recon_status s);
const char* recon_last_error(void);

/* Creates a handle for one geometry, M = `subsets` equal-interval subsets
 * (section 3.D, 1 <= M <= n_views) and TV weight `beta` >= 0 (the alpha of
 * Eq. 2; the update uses beta / M, section 3.D).  params NULL selects the
 * defaults.  Builds the ray tables on the host in double precision, uploads
 * them to the current HIP device and allocates the handle's workspace.  Blocks
 * until the upload has finished.  *out receives the handle. */
recon_status recon_create(const recon_geometry* geom, int32_t subsets, double beta,
                          const recon_params* params, recon_handle** out);

/* Frees the handle, its device tables, workspace and cached graphs.
 * Synchronises the device first.  NULL is accepted. */
recon_status recon_destroy(recon_handle* h);

/* Joseph forward projection (section 4.C "reprojection"): d_sino = A d_img for
 * the views of `subset` (-1 = all), in the order defined above.  d_img is
 * [n][n] in 1/mm, d_sino is [n_sel][n_channels] line integrals
 * (dimensionless).  A ray with |cos| >= |sin| of its direction is sampled once
 * per image column, else once per row; each sample linearly interpolates the
 * two nearest pixels across the sampling line and is weighted by the path
 * length per column (row), pixel_mm / |cos| (|sin|); pixels outside the image
 * are zero. */
recon_status recon_project(recon_handle* h, const float* d_img, float* d_sino, int32_t subset, void* stream);

/* Matched backprojection: d_img = A^T d_sino (overwrites d_img), the exact
 * transpose of recon_project for the same subset, computed per pixel with
 * no atomics (deterministic).  The likelihood gradient of section 2 is
 * A^T (exp(-A mu) - y / I0). */
recon_status recon_backproject(recon_handle* h, const float* d_sino, float* d_img, int32_t subset, void* stream);

/* Gradient of the TV prior: d_grad = -dTV/dmu for
 * TV(mu) = sum_r sqrt(dx_r^2 + dy_r^2 + eps^2), forward differences
 * dx = mu[j][i+1] - mu[j][i], dy = mu[j+1][i] - mu[j][i], zero past the last
 * column / row, eps = tv_eps_per_mm.  Dimensionless, [n][n]. */
recon_status recon_tv_grad(recon_handle* h, const float* d_img, float* d_grad, void* stream);

/* Runs n_iter ordered-subset sub-iterations (one sub-iteration = one
 * "iteration" of the paper: one subset s = n mod M):
 *   f_n      = mean over the subset's rays of (l_i - p_i)^2, l = A_s mu^(n),
 *              p = ln(I0 / max(y, 1))                     (section 3.C.2)
 *   lambda_n = lambda_0 at n = 0, else lambda_{n-1} + lambda_inc if
 *              f_n < f_{n-1}, else lambda_{n-1} - lambda_dec; floor lambda_min
 *                                                          (Eqs. 4-5)
 *   mu^(n+1) = mask * max(0, mu^(n) + lambda_n [A_s^T (exp(-l) - y/I0)
 *              + (beta/M) (-dTV/dmu)])   in cm and 1/cm    (Eq. 3)
 * d_counts: [n_views][n_channels] transmission counts y (natural view order);
 * i0: blank-scan counts (> 0).  d_img: in = mu^(n_done) in 1/mm (pass the
 * homogeneous start from recon_initial_image for a fresh run), out = the
 * final iterate; the start is taken as zero outside the reconstruction disc,
 * where the iterate is held at zero.  state: NULL = fresh run (nothing returned), else read and
 * updated (blocks until the run has finished).  d_trace: NULL or device
 * double [n_iter][2] receiving (f_n, lambda_n).  d_lambda_schedule: NULL or
 * device double [n_iter] replacing the step rule (a replay hook for parity
 * checks; f is still computed).  Sub-iterations are replayed from cached
 * HIP graphs, one per subset epoch.  Returns RECON_NUMERIC when state is
 * given and a non-finite squared difference was met. */
recon_status recon_os_iterate(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                              recon_state* state, double* d_trace, const double* d_lambda_schedule,
                              void* stream);

/* recon_os_iterate with the two step-rule options of recon_params:
 * d_f_hist: NULL or device double [M], in/out: the f of each subset's latest
 *   sub-iteration, read by lambda_compare = 1.  A fresh run needs none (the
 *   handle's own buffer is used when NULL); a resumed run (state->n_done > 0)
 *   with lambda_compare = 1 and M > 1 must pass the array the earlier calls
 *   filled (RECON_INVALID_ARG otherwise).
 * d_best: device float [n][n], 1/mm; required when keep_best = 1 and must be
 *   NULL otherwise (RECON_INVALID_ARG).  Written when an epoch ends with a new
 *   least sum (state->best_n reports which iterate it holds); left untouched
 *   otherwise, so a resumed run passes the same buffer.
 * Every other argument is as for recon_os_iterate, which is this call with
 * both pointers NULL. */
recon_status recon_os_iterate_ex(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                                 recon_state* state, double* d_trace, const double* d_lambda_schedule,
                                 double* d_f_hist, float* d_best, void* stream);

/* Writes the homogeneous start image (section 3.C.2): mu0_per_mm inside the
 * reconstruction disc, 0 outside. */
recon_status recon_initial_image(recon_handle* h, float* d_img, void* stream);

/* Filtered backprojection, the baseline the paper compares the iterative
 * method with (sections 1 and 4; the paper gives no details, so this is the
 * textbook equiangular fan-beam algorithm over the full turn):
 *   p = ln(I0 / max(y, 1)),  R' = p D cos(gamma_k)  (D = sad_mm),
 *   Q = R' convolved per view with dgamma h,  h(0) = 1 / (8 dgamma^2),
 *       h(m) = 0 for even m, -1 / (2 pi^2 sin^2(m dgamma)) for odd m,
 *   f(x, y) = (2 pi / n_views) sum over views of Q(gamma') / L^2,
 * gamma' being the fan angle and L the source distance of (x, y), with Q
 * linearly interpolated in gamma and zero outside the channels.  d_counts:
 * [n_views][n_channels] as for recon_os_iterate; d_img: [n][n] in 1/mm,
 * overwritten, every pixel (no mask).  Deterministic (no atomics).  Uses the
 * handle's workspace: do not overlap with other calls on the same handle.
 * RECON_INVALID_ARG for more than 16384 channels, or for a handle whose views
 * cover less than a full turn (a partial arc would need redundancy weights,
 * which the comparison method is not stated to use). */
recon_status recon_fbp(recon_handle* h, const float* d_counts, float i0, float* d_img, void* stream);

/* Helical rebinning: single-row helical fan data (a helical tomotherapy MVCT
 * scan, section 1) -> one full-turn fan sinogram per slice position, by
 * 360-degree linear interpolation along z (the textbook 360LI method; the
 * paper reconstructs helical MVCT slices but does not state its rebinning).
 * g: the geometry of one turn (n_views views per turn, n_channels channels;
 * scan_arc_rad must be 0 or 2 pi; the other fields are not used).  Helical view h (0 <= h < n_helical_views)
 * has the angle of view h mod n_views and source z = z0_mm + pitch_mm h /
 * n_views (pitch_mm: table feed per turn, > 0).  For slice z and view v the
 * two helical views at that angle whose z bracket z (z_a <= z < z_b) are
 * interpolated with weight w = (z - z_a) / pitch on the measured line
 * integrals l = ln(I0 / max(y, 1)), and the result is written as counts
 * I0 exp(-l), the input form of recon_os_iterate (I0 cancels: the value is
 * y0^(1-w) y1^w with y0, y1 the bracketing counts floored at 1; i0 is
 * validated only).  Bracket, weight and interpolation are in double precision.
 * d_counts: device float [n_helical_views][n_channels]; z_slices: host
 * double [n_slices] (mm); d_out: device float [n_slices][n_views][n_channels],
 * overwritten.  RECON_INVALID_ARG for NULL buffers, non-positive sizes, pitch
 * or I0, or a slice outside [z0 + pitch (n_views - 1) / n_views,
 * z0 + pitch (n_helical_views - n_views) / n_views) (no helical view on one
 * side); nothing is launched then.  n_slices = 0 does nothing. */
recon_status recon_rebin_helical(const recon_geometry* g, int32_t n_helical_views, double pitch_mm, double z0_mm,
                                 const float* d_counts, float i0, const double* z_slices, int32_t n_slices,
                                 float* d_out, void* stream);

/* Data consistency of an image against the counts of the views of every
 * subset_stride-th subset (subsets 0, K, 2K, ... with K = subset_stride; K = 1:
 * every view; for K dividing the subset count, every K-th view of the turn):
 *   d_out[0] = mean over those rays of (l_i - p_i)^2, l = A mu (d_img, 1/mm),
 *              p = ln(I0 / max(y, 1))  (the squared difference of section
 *              3.C.2 taken over those views instead of one subset);
 *   d_out[1] = mean over the same rays of 1 / max(y, 1), the variance of p
 *              under Poisson noise to first order: the level d_out[0] settles
 *              near once the image explains the data.
 * 1 <= subset_stride <= subsets and, for subset_stride > 1, at most 64
 * subsets chosen, else RECON_INVALID_ARG.  d_out: device double[2].  Uses the handle's workspace:
 * do not overlap with other calls on the same handle. */
recon_status recon_data_residual(recon_handle* h, const float* d_counts, float i0, const float* d_img,
                                 int32_t subset_stride, double* d_out, void* stream);

/* Geometry queries (host, synchronous). */
recon_status recon_subset_size(recon_handle* h, int32_t subset, int32_t* n_views_out);

/* Launch shapes are chosen by the library (a new handle uses 16 threads per
 * projector ray from 384^2 images up, 8 from 192^2, else 4, and bp_variant 6);
 * this pins them for tuning and tests.  fp_segments: threads sharing one ray in the projector, in
 * {1, 2, 4, 8, 16}.  bp_variant: 1 = one pixel per thread, candidates read
 * from global memory; 2 = one pixel per thread, candidates staged per 16x16
 * tile in LDS; 3, 4, 5 = LDS-staged with 1x2, 2x1, 2x2 pixels per thread;
 * 6 = LDS-staged with 2x2 pixels per thread and the views split over the four
 * waves of a tile.  0 keeps the current value.  Every choice gives bitwise
 * identical results (each pixel sums its views in four interleaved groups,
 * added in a fixed order).
 * Cached graphs are dropped. */
recon_status recon_set_launch(recon_handle* h, int32_t fp_segments, int32_t bp_variant);


/* ------------------------------------------------------------------------
 * Batches of slices (the many slices of a helical scan, each with its own
 * image size, view count, channel count and I0).  All slices share the subset
 * count M, beta and params.  One sub-iteration of every slice runs as one
 * projector launch, one step-rule launch (a block per slice) and one update
 * launch over work tables that cover all slices; each subset epoch is
 * replayed from a captured HIP graph.  The tables place each slice on one of
 * the 8 XCDs (its data for that kernel then stays in one L2), the update's by
 * its cost (pixels x views) and the projector's by its own (ray samples);
 * when whole slices cannot be balanced within 3 % (fewer slices than XCDs, a
 * few large ones), the largest are cut into 2, 4 or 8 parts placed the same
 * way.  Every slice's result is bitwise equal to recon_os_iterate on that
 * slice alone (fresh state), whatever the placement.
 * ------------------------------------------------------------------------ */
typedef struct recon_batch_handle recon_batch_handle;

/* Creates a batch of n_slices geometries (host array) with M = subsets and
 * TV weight beta (params NULL = defaults): builds every slice's tables and
 * workspace on the current device and the batch's work tables.  Blocks until
 * done. */
recon_status recon_batch_create(const recon_geometry* geoms, int32_t n_slices, int32_t subsets, double beta,
                                const recon_params* params, recon_batch_handle** out);
recon_status recon_batch_destroy(recon_batch_handle* b);

/* Writes every slice's homogeneous start image (as recon_initial_image) into
 * d_imgs, a host array of n_slices device pointers. */
recon_status recon_batch_initial_images(recon_batch_handle* b, float* const* d_imgs, void* stream);

/* Runs n_iter sub-iterations of every slice from a fresh state.  d_counts,
 * d_imgs, d_traces are HOST arrays of n_slices DEVICE pointers: counts
 * [n_views][n_channels] of slice i, image [n][n] of slice i (in: start image,
 * out: result), trace [n_iter][2] of slice i or NULL (d_traces itself may be
 * NULL).  i0 is a host array of n_slices blank-scan counts.  Asynchronous. */
recon_status recon_batch_run(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                             int32_t n_iter, double* const* d_traces, void* stream);

/* Autotuner: times the batched projector for 4, 8 and 16 threads per ray and
 * the batched update for every backprojector variant (reps launches each, on
 * the batch's own data, from the images in d_imgs, which are not modified),
 * keeps the fastest of each for later runs and reports them.  Every choice
 * gives bitwise identical results.  Blocks until done. */
recon_status recon_batch_tune(recon_batch_handle* b, const float* const* d_counts, const float* i0, float* const* d_imgs,
                              int32_t reps, int32_t* fp_segments_out, int32_t* bp_variant_out, void* stream);

/* Pins the batch's launch shapes (as recon_set_launch; 0 keeps).  A new batch
 * starts with bp_variant 6 (2x2 pixels per thread, views split over a tile's
 * waves) and 4 threads per projector ray, the tuner's choice for batches of
 * 512^2 slices, doubled up to 16 while a subset's rays over the whole batch
 * would give the GPU fewer than 2048 threads per compute unit (a batch of one
 * or two 512^2 slices starts at 16). */
recon_status recon_batch_set_launch(recon_batch_handle* b, int32_t fp_segments, int32_t bp_variant);

/* Host-only check of the batched kernels' work tables (no GPU needed): builds,
 * for the given slices, the XCD placement and the tables the batch would
 * upload (the update's 16x16 tiles, the projector's blocks of 256 / fp_segments
 * rays for every subset and for all views) and counts in *errors every tile or
 * ray block that is missing, repeated, out of range or placed on an XCD other
 * than the one its slice, or its part of the slice, is placed on by that
 * kernel's placement (block p runs on XCD p mod 8), and every slice cut into a
 * number of parts other than 1, 2, 4 or 8; *blocks receives the total table length, idle entries included.  RECON_INVALID_ARG as recon_batch_create, or for an
 * fp_segments outside {1, 2, 4, 8, 16}. */
recon_status recon_batch_check_work(const recon_geometry* geoms, int32_t n_slices, int32_t subsets,
                                    int32_t fp_segments, int64_t* errors, int64_t* blocks);

/* One-shot form: create, run n_iter sub-iterations, wait, destroy. */
recon_status recon_batch(const recon_geometry* geoms, int32_t n_slices, int32_t subsets, double beta,
                         const recon_params* params, const float* const* d_counts, const float* i0,
                         float* const* d_imgs, int32_t n_iter, void* stream);

/* Learned warm start for a batch (the network is declared in recon_cnn.h):
 *   1. every slice runs n_pre sub-iterations from the homogeneous start;
 *   2. the network maps each early iterate to an estimate of the converged
 *      image, projected onto the constraints (zero outside the disc,
 *      non-negative); its max_n must cover every slice;
 *   3. n_refine sub-iterations refine that image with a fresh step-rule state
 *      (lambda_0, subsets from 0);
 *   4. the residual r and noise level v of each result are taken as in
 *      recon_data_residual over the views of every check_stride-th subset
 *      (1: every view; same limits as its subset_stride);
 *   5. every slice with r > residual_ratio * v (the level the plain iteration
 *      reaches, calibrated on its own images with the same check_stride) is
 *      reconstructed again from the homogeneous start with n_cold
 *      sub-iterations (alone when one slice falls back, else as a batch).
 * d_counts, d_imgs: host arrays of device pointers as in recon_batch_run
 * (d_imgs receive the results); i0: host array.  h_residual, h_floor (host
 * double[n_slices]) and h_fallback (host int32[n_slices], 1 = cold start used)
 * may be NULL.  Blocks until done (the fallback decision is taken on the
 * host).  Its device staging (the images of one size for the network, the
 * residuals, the count pointers) is allocated by the first call on a batch
 * and kept with the batch for later calls (freed by recon_batch_destroy);
 * calls on one batch must not overlap. */
struct recon_cnn;
recon_status recon_warm_start(recon_batch_handle* b, struct recon_cnn* net, const float* const* d_counts,
                              const float* i0, float* const* d_imgs, int32_t n_pre, int32_t n_refine, int32_t n_cold,
                              double residual_ratio, int32_t check_stride, double* h_residual, double* h_floor,
                              int32_t* h_fallback, void* stream);

/* recon_warm_start for a stream of batches (paper §3.C-§3.D pipeline, as
 * recon_warm_start; a serving loop's form of it): the same arguments, the same
 * results bit for bit and the same fallback decision, but the cold starts of
 * the slices that fall back are enqueued on a stream the batch owns (created
 * by the first such call, default priority), ordered after the check on
 * `stream` by an event, and the call returns once they are enqueued, so that
 * the caller's next batch on `stream` overlaps them.  h_residual, h_floor and
 * h_fallback are filled before it returns; the images of fallback slices are
 * final only once recon_batch_wait(b) has returned.  Every other call on the
 * batch, and recon_batch_destroy, first waits for them.  Allocates like
 * recon_warm_start, plus the stream and two events once per batch. */
recon_status recon_warm_start_async(recon_batch_handle* b, struct recon_cnn* net, const float* const* d_counts,
                                    const float* i0, float* const* d_imgs, int32_t n_pre, int32_t n_refine,
                                    int32_t n_cold, double residual_ratio, int32_t check_stride, double* h_residual,
                                    double* h_floor, int32_t* h_fallback, void* stream);

/* Blocks until the cold starts that recon_warm_start_async left running on
 * the batch are done (returns at once when there are none).
 * RECON_INVALID_ARG for a NULL batch. */
recon_status recon_batch_wait(recon_batch_handle* b);

/* recon_warm_start for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments and the same results, bit for bit, with no hipMalloc,
 * hipFree or graph instantiation during the call.  Its staging buffers live
 * in a fixed scratch array of 16.1 MiB per GPU, reserved in device memory by
 * the library (each GPU it runs on holds it until the process ends): the
 * images pass through the network in chunks of at most 16 MiB, epoch graphs
 * are replayed only if an earlier call on the same batch built them (else the
 * sub-iterations are launched directly), and fallback slices run one by one
 * on their own handles.  Limits: at most 4096 slices per call and images of
 * at most 2048 x 2048; beyond them RECON_INVALID_ARG, with nothing launched.
 * The batch's device must be the current device.  Every call on one GPU
 * shares that GPU's scratch: calls that overlap in time on one GPU (from
 * several threads or on several streams) race and must be serialised by the
 * caller.  No part of the scratch needs to start at zero; each region is
 * written before it is read within a call.  Blocks until done, as
 * recon_warm_start. */
recon_status recon_warm_start_noalloc(recon_batch_handle* b, struct recon_cnn* net, const float* const* d_counts,
                                      const float* i0, float* const* d_imgs, int32_t n_pre, int32_t n_refine,
                                      int32_t n_cold, double residual_ratio, int32_t check_stride, double* h_residual,
                                      double* h_floor, int32_t* h_fallback, void* stream);

/* Number of (ray, in-image pixel) interpolation pairs of `subset` (-1 = all
 * views): the pixel reads of the projector and the sinogram reads of the
 * backprojector, from the handle's own ray tables.  disc_only = 1 counts only
 * pairs whose pixel lies in the reconstruction disc (the pixels where an
 * iteration's iterate can be nonzero).  Host, synchronous. */
recon_status recon_count_pairs(recon_handle* h, int32_t subset, int32_t disc_only, int64_t* pairs);

/* Measurement helper (no operation of the paper): the read bandwidth the cache
 * hierarchy delivers to a kernel that gathers from a buffer held in L2, as a
 * ceiling for the gather kernels' algorithmic rates.  2048 blocks of 256
 * threads (8 per compute unit) each read all of a `bytes`-byte buffer (a power
 * of two in [16 KiB, 64 MiB]; 2 MiB fits the 4 MB L2 of every XCD) with
 * 16-byte loads, after one untimed launch that brings it into the caches;
 * *gbps_out = bytes read / time over `reps` (1..100) launches timed with HIP
 * events on `stream`.  Allocates and frees its own buffers; blocks until done.
 * RECON_INVALID_ARG for other sizes or counts. */
recon_status recon_read_bandwidth(int64_t bytes, int32_t reps, double* gbps_out, void* stream);

/* Measurement helper (no operation of the paper): the vector ALU's issue rate
 * for one instruction, as a check of the ALU ceiling the gather kernels are
 * measured against.  2048 blocks of 256 threads (8 waves per SIMD) each run 16
 * independent chains of 1024 instances of the instruction `op`: 0 v_fmac_f32
 * (sources in two different registers), 1 v_add_f32, 2 v_add_u32,
 * 3 v_cvt_f32_i32, 4 v_lshl_add_u64, 5 v_dot2c_f32_bf16.  *lane_ops_out = lane
 * operations per second (wave64 instructions x 64) over `reps` (1..100)
 * launches timed with HIP events on `stream`, after one untimed launch.
 * Allocates and frees its own buffers; blocks until done.  RECON_INVALID_ARG
 * for other ops or counts. */
recon_status recon_valu_rate(int32_t op, int32_t reps, double* lane_ops_out, void* stream);

/* Measurement helper: from d_img (read only) runs one sub-iteration of every
 * subset, then launches each kernel of a sub-iteration n_iter (1..4096) times
 * back to back on `stream` (subsets in turn) between two HIP events, and
 * writes the mean time per launch in ms of the projector to ms_out[0] and of
 * the fused step-rule + backprojection + update kernel to ms_out[2]
 * (ms_out[1] = 0: the step rule has no launch of its own).  Then it runs
 * min(n_iter, 256) sub-iterations' kernels in their order (projector, update,
 * subsets in turn) with a pair of HIP events around every launch, and writes
 * the mean of the update's launches to ms_out[3] and of the projector's to
 * ms_out[4] (each kernel then meets the cache state the other leaves, as in a
 * reconstruction).  ms_out: 5 doubles.  Blocks until done. */
recon_status recon_time_kernels(recon_handle* h, const float* d_counts, float i0, float* d_img, int32_t n_iter,
                                double* ms_out, void* stream);

/* Host-only self-check of the ray tables (no GPU needed): for every
 * view_stride-th view and every pixel, counts the (pixel, ray) pairs with a
 * nonzero interpolation weight that the backprojector's candidate windows
 * (the per-pixel windows and the per-tile linear windows of the LDS-staged
 * gather) would miss (*missed, must be 0), the per-pixel candidates (*candidates) and
 * the nonzero pairs (*pairs); also counts into *missed projector samples
 * outside a ray's stored sample range and per-tile windows outside the
 * channel range the staged gather holds in LDS. */
recon_status recon_check_tables(const recon_geometry* geom, int32_t subsets, int32_t view_stride, int64_t* missed,
                                int64_t* candidates, int64_t* pairs);

#ifdef __cplusplus
}
#endif

#endif /* RECON_H */
