/*
 * clean.h -- C ABI of the MI355X (gfx950) Hogbom CLEAN library.
 *
 * Operations (Wright, Adamek, Armour, "Distribution of the Hogbom CLEAN
 * Algorithm Using Tiled Images with Feedback", arXiv 2501.01461):
 *
 *   clean_hogbom          the Hogbom minor loop (Section 3, the two update
 *                         equations): find the pixel of largest |residual|,
 *                         append (position, gain * value) to the component
 *                         list, subtract gain * value * PSF centred there.
 *   clean_tiled_feedback  the tiled form with feedback (Sections 2 and 3,
 *                         Figs. 1-3): tiles run their own minor loops on their
 *                         own pixels; at a fixed interval each tile's new
 *                         components, convolved with the full PSF (the
 *                         cross-coupling image), are subtracted from every
 *                         other tile.
 *   clean_batched         many independent Hogbom problems of uneven size, each
 *                         with its own PSF, in one persistent launch (not in the
 *                         paper; a serving form of the same minor loop).
 *   clean_psf_to_f16      converts an FP32 PSF to FP16 storage (round to
 *                         nearest even) for the half-traffic PSF option.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are row-major float32, ny rows of nx pixels; a pixel's index is
 *   y * nx + x.  The PSF is row-major, psf_ny x psf_nx with psf_ny >= 2*ny and
 *   psf_nx >= 2*nx, its centre (peak) at (psf_ny/2, psf_nx/2).  Subtracting the
 *   PSF "centred on p" updates pixel q with psf[q - p + centre]; with the size
 *   rule no index ever leaves the PSF.
 * - Unless stated, every pointer argument is a DEVICE pointer (memory from
 *   hipMalloc or a torch CUDA tensor on the current device) and the CALLER owns
 *   it; the library never frees caller memory.  `clean_params`, `clean_stats`
 *   and `clean_problem` arrays are HOST memory.
 * - `stream` is a hipStream_t (NULL = the default stream).  Work is queued on
 *   it, and every call synchronises the stream before it returns (the stats
 *   need the device's counters), so calls are synchronous.
 * - Return value: CLEAN_OK, or a negative clean_status.  Arguments are checked
 *   before anything is launched; on an argument error nothing is written.
 *   clean_last_error() gives a thread-local message for the last failure.
 * - Arithmetic (the FP32 path): component = fl32((float)gain * v); each pixel
 *   update is one fused multiply-add r = fma(-component, psf, r); the peak is
 *   the largest |r| with ties going to the lowest index; the stop tests, made
 *   before each append, are n == max_iter, then v not finite, then
 *   (double)|v| < threshold, then n == capacity.  IEEE subnormals are kept.
 *   With an FP32 PSF the plain path's components and residual are
 *   bit-identical to a serial CPU run of the same definition.
 * - Non-finite values: the peak search orders |r| with +Inf above every
 *   finite value and every NaN above +Inf (all NaNs equal, lowest index
 *   first), so a region holding a NaN or an infinity has a non-finite peak,
 *   and a non-finite peak ends the run with CLEAN_STOP_NONFINITE before
 *   anything is appended.  This covers a run that diverges (values overflow)
 *   as well as non-finite input: with CLEAN_FLAG_CHECK_FINITE the dirty image
 *   and the PSF are scanned first and CLEAN_E_NONFINITE is returned instead.
 * - Concurrency: calls that use the library's internal workspace (workspace ==
 *   NULL) must not overlap on one device; pass separate workspaces to overlap.
 */
#ifndef CLEAN_H
#define CLEAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CLEAN_OK = 0,
    CLEAN_E_INVAL = -1,       /* bad argument (message in clean_last_error)   */
    CLEAN_E_NONFINITE = -2,   /* NaN/Inf found with CLEAN_FLAG_CHECK_FINITE   */
    CLEAN_E_NOMEM = -3,       /* workspace allocation failed / too small      */
    CLEAN_E_HIP = -4,         /* a HIP runtime call failed                    */
    CLEAN_E_TIMEOUT = -5,     /* a device-side wait exceeded its time limit   */
    CLEAN_E_UNSUPPORTED = -6  /* shape or option outside what is implemented  */
} clean_status;

typedef enum {
    CLEAN_STOP_MAXITER = 0,   /* max_iter components were found               */
    CLEAN_STOP_THRESHOLD = 1, /* every peak is below the threshold            */
    CLEAN_STOP_CAPACITY = 2,  /* comp_cap components were found first         */
    CLEAN_STOP_CANCELLED = 3, /* the caller's cancel flag was set             */
    CLEAN_STOP_NONFINITE = 4  /* a peak was NaN or infinite (the run diverged,
                                 or non-finite input was not screened out)    */
} clean_stop;

typedef enum { CLEAN_PSF_F32 = 0, CLEAN_PSF_F16 = 1 } clean_psf_dtype;

enum {
    CLEAN_FLAG_CHECK_FINITE = 1,   /* scan inputs for NaN/Inf before starting      */
    CLEAN_FLAG_STREAM_RESIDUAL = 2,/* keep the residual in HBM even when it would
                                      fit the register file (plain and tiled)     */
    CLEAN_FLAG_FFT_FEEDBACK = 4,   /* tiled: after each round, compute the
                                      residual as the round's starting residual
                                      minus one FFT convolution of all the
                                      round's components with the PSF (the same
                                      update as the direct gather, own tile
                                      included); images up to 32768 x 32768.
                                      Not bit-identical to the direct form:
                                      float32 transforms, relative error ~1e-6
                                      of the convolution's scale per round.
                                      Workspace grows by about
                                      (3 Hx R + Hx Ly) * 8 + ny nx * 4 bytes,
                                      Lx, Ly the powers of two >= 2 nx - 1,
                                      2 ny - 1, Hx = Lx/2 + 1, R = max(ny, Ly);
                                      axes longer than 8192 points add two-level
                                      work buffers (clean_workspace_size)      */
    CLEAN_FLAG_FFT_TWO_LEVEL = 8   /* with CLEAN_FLAG_FFT_FEEDBACK: use the
                                      two-level (four-step) transforms on every
                                      axis of length >= 4, as they are used
                                      automatically above 8192 points (slower;
                                      for testing that path at small sizes)    */
};

typedef struct {
    double gain;          /* loop gain, 0 < gain <= 1 (applied as float)          */
    double threshold;     /* Jy; stop when |peak| < threshold; >= 0               */
    int64_t max_iter;     /* total minor iterations (all tiles together); >= 0    */
    int32_t psf_dtype;    /* clean_psf_dtype of the `psf` argument                */
    int32_t flags;        /* CLEAN_FLAG_* bits                                    */
    int32_t wg_per_tile;  /* launch shape: workgroups per tile (0 = library pick) */
    int32_t px_per_thread;/* launch shape: residual pixels per thread, one of
                             4, 8, 16, 32, 64 when tile widths are multiples of
                             4, else 4, 16, 32 (0 = library pick).  Tiled calls
                             also take 128: the wide tile (one workgroup per
                             CU, residual in registers during the local loops
                             only), which the library picks by itself for
                             tiles too large for the other shapes; it needs
                             equal tile widths, multiples of 4, dividing
                             2048 x (its workgroups per tile), and
                             wg_per_tile = 0                                   */
    double feedback_level;/* tiled only, in [0, 1]: the flux trigger.  Each
                             round's level is this fraction of the largest tile
                             peak at the round's start; a tile takes part only
                             if its peak is at or above the level and ends its
                             round when its peak drops below it (or after
                             feedback_interval iterations).  0 = interval only */
    const volatile int32_t *cancel; /* NULL, or a flag in host memory the
                             device can read (hipHostMalloc'ed, or pinned by
                             torch), written by another host thread while the
                             call runs.  Once it holds a non-zero value the run
                             stops at its next checkpoint with
                             CLEAN_STOP_CANCELLED: plain and batched problems
                             every 4096 iterations (iteration 0 included),
                             tiled runs at each round's start.  The results are
                             then those of the same call with max_iter = the
                             iterations done.  A checkpoint costs one extra
                             peak exchange (plain) and one read of host memory */
} clean_params;

typedef struct {
    int64_t n_iter;       /* components written                                   */
    int32_t stop_reason;  /* clean_stop                                           */
    int32_t n_rounds;     /* feedback rounds (tiled); 0 for plain                 */
    double final_peak;    /* signed value of the largest |residual| at the stop   */
    double residual_rms;  /* sqrt(mean(residual^2)), float64 accumulation         */
    double model_flux;    /* sum of all components, float64 accumulation          */
    float device_ms;      /* device time of the call (HIP events)                 */
    int32_t wg_per_tile;  /* launch shape that was used                           */
    int32_t px_per_thread;
    int32_t workgroups;   /* total workgroups in the persistent launch            */
    float phase_us[3];    /* tiled: device time in the local loops, the feedback
                             gather and the apply + re-peak phases, summed over
                             rounds (microseconds, wall clock); 0 for plain       */
    int32_t streamed;     /* 1: the residual was kept in HBM (image too large for
                             the register file of the co-resident workgroups);
                             0: held in registers for the whole run              */
    int32_t xcd_local_clusters; /* clusters whose per-iteration peak exchange
                             stayed inside one XCD's L2 (all their workgroups
                             ran on one XCD, checked on the device); the others
                             used device-scope exchanges.  Tiled: tile clusters
                             counted; batched: 1 or 0 for that problem; plain:
                             0                                                   */
    int32_t exchange_levels; /* plain: 2 when the cluster's per-iteration
                             exchange ran in two levels (keys gathered inside
                             each XCD first, then across the 8 XCD leaders;
                             clusters of 32 or more workgroups placed one
                             rank per XCD in turn, checked on the device),
                             else 1; tiled and batched: 1                     */
} clean_stats;

/*
 * clean_hogbom -- plain Hogbom CLEAN on one image (Section 3, eqs. 1 and 2).
 *
 *   dirty      [ny*nx] float32 input image; may alias `residual` (in place).
 *   psf        [psf_ny*psf_nx] float32, or float16 bits when
 *              p->psf_dtype == CLEAN_PSF_F16 (values are widened to float32
 *              before the fma).
 *   residual   [ny*nx] float32 output.
 *   comp_idx   [comp_cap] int32 output: pixel index of component k, in the
 *              order found.
 *   comp_flux  [comp_cap] float32 output: component value k.
 *   model      [ny*nx] float64 output or NULL: per-pixel sum of components in
 *              list order.
 *   workspace  device scratch of workspace_bytes (>= clean_workspace_size()),
 *              or NULL to use a library-owned buffer.
 *   stats      host output, may be NULL.
 * Limits: ny*nx <= 2^28; ((ny-1)*psf_nx + nx) * element size < 2^32.
 * Images whose residual fits the register file of the co-resident workgroups
 * keep it there for the whole run; larger ones stream it through `residual`.
 */
int clean_hogbom(const float *dirty, int ny, int nx,
                 const void *psf, int psf_ny, int psf_nx,
                 const clean_params *p,
                 float *residual,
                 int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                 double *model,
                 void *workspace, size_t workspace_bytes,
                 clean_stats *stats, void *stream);

/* Size of the device scratch array behind clean_hogbom_noalloc, per GPU. */
#define CLEAN_NOALLOC_SCRATCH_BYTES 65536

/*
 * clean_hogbom_noalloc -- clean_hogbom for callers that cannot allocate
 * memory in the call: code that must not call hipMalloc (tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * errors as clean_hogbom without a workspace argument: the call allocates
 * nothing (no device, pinned or stream-ordered allocation, no events).  Its
 * workspace is a file-scope device array of CLEAN_NOALLOC_SCRATCH_BYTES bytes,
 * one copy per GPU, held until the process ends; its device address is looked
 * up once per device, on the first call there.  Every call on a GPU shares
 * that GPU's array: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller; the control words the
 * kernels need zeroed are cleared by a fill kernel at the start of each call.
 * A launch shape whose workspace exceeds the array (a cluster of more than
 * about 1000 workgroups, which only a forced wg_per_tile can ask for: the
 * library's launches hold at most two workgroups per CU) fails with
 * CLEAN_E_UNSUPPORTED before anything is launched.  stats->device_ms is 0 (the call is not timed).  Synchronous, as
 * every entry point.
 */
int clean_hogbom_noalloc(const float *dirty, int ny, int nx,
                         const void *psf, int psf_ny, int psf_nx,
                         const clean_params *p,
                         float *residual,
                         int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                         double *model,
                         clean_stats *stats, void *stream);

/*
 * clean_tiled_feedback -- tiled Hogbom CLEAN with feedback (Sections 2-3).
 *
 * Tiles: tile (i, j), id i*tiles_x + j, covers rows [i*ny/tiles_y,
 * (i+1)*ny/tiles_y) and columns [j*nx/tiles_x, (j+1)*nx/tiles_x) (floor
 * division).  Each round: tiles whose peak is >= threshold are active; each
 * active tile runs up to `feedback_interval` minor iterations on its own pixels
 * (with p->feedback_level > 0, a tile is active only at or above the round's
 * flux level and its round also ends when its peak falls below it)
 * (when fewer than |active| * interval iterations remain, the remainder is split
 * evenly, lower tile ids taking the extra one); then every tile's new
 * components are placed on a component image (float64 sums in the order found,
 * rounded once to float32) and, for every pixel q of tile s,
 *   acc = 0;  for every other tile t in ascending order, for each of its
 *   non-zero component pixels c in row-major order:
 *             acc = fmaf(value_c, psf[q - c + centre], acc);
 *   r[q] = r[q] - acc.
 * The run stops at the start of a round when max_iter components exist, when
 * the cancel flag is set, when a tile's peak is not finite
 * (CLEAN_STOP_NONFINITE), when no tile is active,
 * or when comp_cap components exist; inside a round a tile's loop also ends
 * at a non-finite peak.  Every round ends with its feedback, so
 * residual + components (*) PSF = dirty holds at return.
 *
 *   comp_idx/comp_flux   order: round, then tile id, then local iteration.
 *   feedback_interval    1 .. 2048.  Without CLEAN_FLAG_FFT_FEEDBACK, a call
 *                        whose direct gather could read more than 2^44 bytes
 *                        of PSF in one round (tiles x interval components,
 *                        each over the pixels outside its tile) is refused
 *                        with CLEAN_E_UNSUPPORTED: that phase could outlast
 *                        the device's wait limit; the FFT form has no such
 *                        bound.
 *   tiles_y, tiles_x     1 .. ny (nx); at most 1024 tiles.
 * Other arguments as for clean_hogbom.  With tiles_y = tiles_x = 1 the result
 * equals clean_hogbom's bit for bit.
 */
int clean_tiled_feedback(const float *dirty, int ny, int nx,
                         const void *psf, int psf_ny, int psf_nx,
                         int tiles_y, int tiles_x, int feedback_interval,
                         const clean_params *p,
                         float *residual,
                         int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                         double *model,
                         void *workspace, size_t workspace_bytes,
                         clean_stats *stats, void *stream);

/*
 * One problem of a batch: the fields mirror clean_hogbom's (or, with a tile
 * grid, clean_tiled_feedback's) arguments (device pointers, caller-owned).
 * threshold, max_iter and the tile grid are per problem; gain, psf_dtype,
 * flags, feedback_level and cancel come from the shared clean_params.
 */
typedef struct {
    const float *dirty;
    const void *psf;
    float *residual;
    int32_t *comp_idx;
    float *comp_flux;
    double *model;        /* may be NULL */
    int64_t comp_cap;
    int64_t max_iter;
    double threshold;
    int32_t ny, nx, psf_ny, psf_nx;
    int32_t tiles_y, tiles_x; /* 0 or 1 x 1: plain Hogbom; else the tiled form
                                 with feedback (direct gather), as
                                 clean_tiled_feedback                         */
    int32_t interval;         /* tiled problems: feedback interval, 1..2048  */
} clean_problem;

/*
 * clean_batched -- n independent Hogbom problems in one persistent launch,
 * each plain or tiled with feedback.  Workgroups take problems from a device
 * queue, those with the most workgroups first: per XCD when every XCD holds
 * the largest problem (each problem then runs on one XCD and its exchanges
 * stay in that XCD's L2), else across the device.  A tiled problem's tiles
 * are clusters of its own workgroups, which also share its feedback gather,
 * with barriers among them only.  Each problem's result is identical to
 * clean_hogbom (or clean_tiled_feedback) on it alone.
 *   probs  host array of n problems; stats host array of n (may be NULL):
 *          n_rounds counts a tiled problem's rounds, wg_per_tile its
 *          workgroups per tile, xcd_local_clusters its clusters that
 *          exchanged inside one XCD.
 * Uses the library's internal workspace; n <= 65536.  A batch holding a
 * tiled problem runs a kernel variant with more registers per thread (one
 * workgroup per CU at 32 px/thread).  CLEAN_FLAG_FFT_FEEDBACK is not
 * supported here (CLEAN_E_UNSUPPORTED); a problem fails validation as
 * clean_tiled_feedback would (message "problem i: ...").
 */
int clean_batched(const clean_problem *probs, int n, const clean_params *shared,
                  clean_stats *stats, void *stream);

/*
 * clean_autotune_batched -- picks the pixels per thread of clean_batched for
 * this batch by timing one trial launch per candidate (8, 16, 32, 64; those
 * that do not fit the batch are skipped) with every problem's max_iter capped
 * at trial_iter, and writes the fastest to *px_per_thread.  The shape does
 * not change any result, only the speed.  The trials overwrite the problems'
 * residual, component and model arrays.  The choice is cached per process by
 * device and batch signature (PSF dtype, flags, and every problem's image,
 * PSF and tile-grid sizes and interval, in order); clean_batched with
 * shared->px_per_thread = 0 then uses it instead of its built-in rule.
 *   trial_ms  host array of CLEAN_BATCH_TUNE_CANDIDATES (may be NULL): each
 *             candidate's launch time in ms, -1 where it did not fit.
 * Errors as clean_batched; CLEAN_E_UNSUPPORTED if no candidate fits.
 */
#define CLEAN_BATCH_TUNE_CANDIDATES 4
int clean_autotune_batched(const clean_problem *probs, int n, const clean_params *shared,
                           int64_t trial_iter, int *px_per_thread, float *trial_ms, void *stream);

/*
 * clean_autotune -- picks the launch shape (p->wg_per_tile, p->px_per_thread)
 * of clean_hogbom (tiles_y = tiles_x = 1) or clean_tiled_feedback for this
 * image, PSF dtype and tile grid by timing trial runs of `trial_iter` minor
 * iterations (capped by p->max_iter) on the caller's buffers, and writes the
 * fastest into *best (a copy of *p with the two shape fields set).  Every
 * shape gives bit-identical results; only the speed differs.  The residual and
 * component arrays are overwritten by the trials.  The choice is cached per
 * process by (device, ny, nx, tile grid, interval, PSF dtype, streaming flag).
 * Arguments otherwise as for clean_tiled_feedback.
 */
int clean_autotune(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                   int tiles_y, int tiles_x, int feedback_interval, const clean_params *p,
                   float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                   int64_t trial_iter, clean_params *best, void *stream);

/*
 * clean_autotune_interval -- picks the feedback interval of
 * clean_tiled_feedback among `candidates` (n_candidates in 1..64, each in
 * 1..2048).  Unlike the launch shape, the interval changes the result (the
 * tiles run longer between feedback rounds), and with a PSF of high
 * sidelobes a long interval can make the method diverge.  Each candidate gets
 * a trial run of min(trial_iter, p->max_iter) total iterations on the
 * caller's buffers (p's flags, trigger level and launch shape apply).  A
 * candidate is acceptable when the trial's residual stays finite and its
 * final peak |residual| is at most growth_limit times the dirty image's peak;
 * the acceptable candidate with the highest iteration rate is written to
 * *interval, or 0 when none is acceptable (status still CLEAN_OK).
 * rate_out / peak_ratio_out (host, n_candidates, may be NULL) receive each
 * trial's iterations per second and final-peak / dirty-peak ratio.  The
 * residual and component arrays are overwritten by the trials.  Errors:
 * CLEAN_E_INVAL for a NULL p or interval, bad candidates, a 1x1 grid,
 * trial_iter < 1 or growth_limit <= 0; otherwise as clean_tiled_feedback.
 */
int clean_autotune_interval(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                            int tiles_y, int tiles_x, const int *candidates, int n_candidates,
                            const clean_params *p, int64_t trial_iter, double growth_limit,
                            float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                            int *interval, double *rate_out, double *peak_ratio_out, void *stream);

/*
 * clean_autotune_plan -- picks the tile grid and the feedback interval of
 * clean_tiled_feedback for this image under an accuracy budget.  The paper
 * (Section 4) reports the tiled result within -0.1 .. +0.04 Jy of plain
 * CLEAN, and the interval and tile count decide whether the method holds it
 * at all (with a PSF of high sidelobes a long interval diverges).  So every
 * candidate pair (grids[2i], grids[2i+1]) x intervals[j] gets a trial run of
 * min(trial_iter, p->max_iter) total iterations on the caller's image, beside
 * one plain clean_hogbom run of the same length; both are restored
 * (clean_beam_fit, clean_restore) and the pair is acceptable when every pixel
 * of restored(tiled) - restored(plain) lies in [band_min, band_max] Jy and
 * the run did not go non-finite.  The acceptable pair with the highest trial
 * rate (minor iterations per second) is written to *plan with its band and
 * its launch shape; plan->interval = 0 when none is acceptable (status still
 * CLEAN_OK).  band_out (host, 2 * n_grids * n_intervals, may be NULL) and
 * rate_out (host, n_grids * n_intervals, may be NULL) get every candidate's
 * band and rate, candidate index = grid index * n_intervals + interval
 * index (NaN for a grid with no launch).
 * cache_path (may be NULL): a text file of plans, one line per key (device
 * architecture and name, image and PSF shape, PSF dtype, flags, gain,
 * threshold, max_iter, trial length, trigger level, budget, candidates).  A
 * key found there is returned without any trial (plan->from_cache = 1): the
 * plan was validated on the image of the call that stored it.  New plans are
 * appended.  The library allocates its trial buffers (about 40 bytes per
 * pixel).  Arguments: 1..16 grids (not 1 x 1) and 1..16 intervals, trial_iter
 * >= 1, band_min <= 0 <= band_max, otherwise CLEAN_E_INVAL; errors of the
 * trial runs are returned as they are.
 */
typedef struct {
    int32_t tiles_y, tiles_x, interval; /* the chosen pair; interval 0: none acceptable */
    int32_t wg_per_tile, px_per_thread; /* the launch shape of its trial                  */
    double band_min, band_max;          /* restored tiled - plain over the image, Jy     */
    double iters_per_s;                 /* the trial's minor iterations per second       */
    int32_t from_cache;                 /* 1: read from cache_path                       */
} clean_plan;

int clean_autotune_plan(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                        const int *grids, int n_grids, const int *intervals, int n_intervals,
                        const clean_params *p, int64_t trial_iter, double band_min, double band_max,
                        const char *cache_path, clean_plan *plan, double *band_out, double *rate_out,
                        void *stream);

/* Bytes of device workspace clean_hogbom (tiles 1x1) or clean_tiled_feedback
 * needs for this shape; 0 on invalid arguments. */
size_t clean_workspace_size(int ny, int nx, int tiles_y, int tiles_x,
                            int feedback_interval, const clean_params *p);

/*
 * Restoration: the "reconstructed image" of the paper's comparison (Section 4)
 * read as the usual restored image, the model convolved with a circular
 * Gaussian clean beam of peak 1, plus the residual.
 *
 * clean_beam_fit -- the clean beam of a PSF (device memory, psf_ny x psf_nx,
 * dtype CLEAN_PSF_F32/F16, centre (psf_ny/2, psf_nx/2)): *area (host) gets the
 * pixel count of the main lobe (the 4-connected region of values above one
 * half containing the centre) and *sigma (host) the beam's standard deviation
 * in pixels, FWHM / (2 sqrt(2 ln 2)) with FWHM = 2 sqrt(area / pi).  Reads a
 * crop about the centre (grown until the lobe stays inside it); synchronous.
 * CLEAN_E_INVAL for NULL pointers, a bad size or dtype, or a centre value not
 * above one half.
 *
 * clean_restore -- out[q] = residual[q] + sum over |dy|, |dx| <= R of
 * model[q - d] exp(-(dy^2 + dx^2) / (2 sigma^2)), R = ceil(5 sigma), pixels
 * outside the image counting as zero.  model and out float64 [ny][nx],
 * residual float32 [ny][nx], all device memory owned by the caller (out must
 * not alias the inputs); computed in float64 as two separable passes (the
 * library's workspace holds the intermediate); synchronous on `stream`.
 * CLEAN_E_INVAL for NULL pointers, a bad size or sigma outside (0, 1000].
 */
int clean_beam_fit(const void *psf, int psf_ny, int psf_nx, int psf_dtype, int64_t *area, double *sigma,
                   void *stream);
int clean_restore(const double *model, const float *residual, int ny, int nx, double sigma, double *out,
                  void *stream);

/* FP32 -> FP16 (round to nearest even) of n values, on `stream`; synchronous. */
int clean_psf_to_f16(const float *psf, uint16_t *out, int64_t n, void *stream);

/*
 * clean_bandwidth_probe -- not part of the method: the memory bandwidth a
 * working set achieves on the current device, the denominators of the
 * kernels' rooflines.  buf: caller-owned device memory of `bytes` bytes
 * (>= 4096, a multiple of 32).  mode 0 reads the buffer `reps` times with
 * 16-byte loads (every workgroup re-reads its own words, so a buffer small
 * enough for the L2s, or for the Infinity Cache, is served from them after
 * the first pass); mode 1 copies the first half onto the second half `reps`
 * times.  *gbs (host) = bytes x reps / kernel time, in GB/s (1e9 B/s): the
 * bytes read (mode 0) or read plus written (mode 1).  Synchronous.
 * CLEAN_E_INVAL for NULL pointers or arguments out of range.
 */
int clean_bandwidth_probe(void *buf, size_t bytes, int mode, int reps, double *gbs, void *stream);

/*
 * clean_set_workspace_limit -- caps the device memory the library allocates
 * for its internal workspace (calls with workspace == NULL, batched calls,
 * restoration): a call that would need more fails with CLEAN_E_NOMEM before
 * anything is launched.  0 removes the cap (the default).  Returns the
 * previous cap.  Applies to every device and thread of the process.
 */
size_t clean_set_workspace_limit(size_t bytes);

/* Static description of a clean_status value. */
const char *clean_strerror(int status);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *clean_last_error(void);

/* Library version string. */
const char *clean_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CLEAN_H */
