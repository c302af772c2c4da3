/*
 * CPU oracle for Hogbom CLEAN and for tiled Hogbom CLEAN with feedback.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against.  It shares no code, header, table or helper
 * with the GPU library, and the GPU library never calls it.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * It is deliberately plain and slow: every step below is the textbook step of
 * the paper (Wright, Adamek, Armour, "Distribution of the Hogbom CLEAN
 * Algorithm Using Tiled Images with Feedback", arXiv 2501.01461), written out
 * in the order the paper gives it, with no blocking, fusion or reordering.
 *
 * Build: cc -O3 -mavx2 -mfma -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 *        (no contraction: every fused multiply-add below is an explicit fma).
 *        OpenMP only splits loops whose iterations touch disjoint pixels with
 *        unchanged per-pixel arithmetic, so any thread count gives the same
 *        bits as one thread; the peak search stays a serial scan.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes; the paper states none of them):
 *   - "highest intensity" is the largest |r|; the component keeps the signed
 *     value.  Ties go to the lowest row-major index.
 *   - component = fl(gain * v), one rounding in the working precision.
 *   - the PSF is at least twice the image on each axis, centred at
 *     (psf_ny/2, psf_nx/2); pixel q gets psf[q - p + centre] (no clipping).
 *   - the subtraction is r = fma(-c, psf, r): one rounding per pixel.
 *   - stop tests, before each append: n == max_iter, then |v| < threshold
 *     (tested in double), then n == capacity.
 *   - tiles: an equal floor split, tile (i, j) covers rows
 *     [i*ny/ty, (i+1)*ny/ty) and columns [j*nx/tx, (j+1)*nx/tx); a tile works
 *     on its own pixels only; every round ends with feedback.
 *   - feedback, per round: each tile's new components are placed on a
 *     full-size component image (per-pixel sums in double, in the order they
 *     were found, then one rounding to the working precision); convolving that
 *     image directly with the full PSF gives the tile's cross-coupling image.
 *     At each pixel the cross-coupling images of all OTHER tiles are summed as
 *     one fma chain from zero (tiles in ascending order, each tile's non-zero
 *     component pixels in raster order) and the sum is subtracted once.
 *   - "total iterations" for the tiled form counts the minor iterations of all
 *     tiles together; per-round budgets split what remains evenly.
 *   - feedback "at regular intervals" is the interval: a tile's round ends
 *     after `interval` local iterations.  Feedback "triggered by meeting a
 *     flux threshold" is the level: with level_frac > 0 a round's flux level
 *     is level_frac times the largest tile peak at the round's start, a tile
 *     takes part only if its peak is at or above it, and its round also ends
 *     when its peak drops below it.
 *   - non-finite values (a run that diverges, or NaN/Inf input that was not
 *     screened out): the peak search orders |r| as IEEE magnitudes with every
 *     NaN above +Inf and all NaNs equal, so the lowest-index NaN, else the
 *     lowest-index infinity, is the peak of a region holding any.  A
 *     non-finite peak ends the run (stop reason "non-finite") before anything
 *     is appended: the plain loop tests it right after n == max_iter; the
 *     tiled form tests every tile's peak at a round's start (after
 *     used == max_iter), and inside a round a non-finite local peak ends that
 *     tile's round like a peak below the threshold does, so the round still
 *     ends with its feedback.  The round's flux level is therefore always a
 *     finite fraction of a finite peak.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -3 };
enum { STOP_MAXITER = 0, STOP_THRESHOLD = 1, STOP_CAPACITY = 2, STOP_NONFINITE = 4 };

static int check_common(int ny, int nx, int psf_ny, int psf_nx, double gain, double threshold,
                        int64_t max_iter, int64_t cap)
{
    if (ny <= 0 || nx <= 0) return OR_EINVAL;
    if (psf_ny < 2 * ny || psf_nx < 2 * nx) return OR_EINVAL;
    if (!(gain > 0.0 && gain <= 1.0)) return OR_EINVAL;
    if (!(threshold >= 0.0) || max_iter < 0 || cap < 0) return OR_EINVAL;
    return OR_OK;
}

/* ---------------------------------------------------------------- FP32 -- */

/* Position of the highest |r| inside the rectangle [y0,y1) x [x0,x1) of a
 * row-major image of width nx: the lowest row-major index whose |r| equals the
 * largest |r| (so the lowest index wins a tie).  Two plain scans: the largest
 * value, then the first pixel holding it.  |r| is compared through its bit
 * pattern: with the sign bit cleared, IEEE-754 values order exactly as their
 * bit patterns read as unsigned integers, +Inf above every finite value.
 * Every NaN is given one magnitude, the quiet NaN's, above +Inf, so a NaN is
 * the peak of any region holding one and the first NaN wins among NaNs. */
static uint32_t mag_f32(float v)
{
    uint32_t b;
    memcpy(&b, &v, sizeof b);
    b &= 0x7FFFFFFFu;
    return b > 0x7F800000u ? 0x7FC00000u : b;
}

static int64_t peak_f32(const float *r, int nx, int y0, int y1, int x0, int x1)
{
    uint32_t best = 0;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            uint32_t a = mag_f32(r[(int64_t)y * nx + x]);
            best = a > best ? a : best;
        }
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x)
            if (mag_f32(r[(int64_t)y * nx + x]) == best) return (int64_t)y * nx + x;
    return (int64_t)y0 * nx + x0;   /* not reached */
}

/* Exposed for the peak-order pin: the peak of a rectangle (-1 if empty). */
int64_t oracle_peak_f32(const float *r, int nx, int y0, int y1, int x0, int x1)
{
    if (nx <= 0 || y0 < 0 || x0 < 0 || y1 <= y0 || x1 <= x0 || x1 > nx) return -1;
    return peak_f32(r, nx, y0, y1, x0, x1);
}

/* r[q] -= c * PSF centred on p, for q in the rectangle (eq. 2 of Section 3). */
static void subtract_psf_f32(float *r, int nx, int y0, int y1, int x0, int x1, int64_t p, float c,
                             const float *psf, int psf_nx, int cy, int cx)
{
    int py = (int)(p / nx), px = (int)(p % nx);
#pragma omp parallel for schedule(static) if ((int64_t)(y1 - y0) * (x1 - x0) > 65536)
    for (int y = y0; y < y1; ++y) {
        const float *prow = psf + (int64_t)(y - py + cy) * psf_nx + (cx - px);
        float *rrow = r + (int64_t)y * nx;
        for (int x = x0; x < x1; ++x)
            rrow[x] = fmaf(-c, prow[x], rrow[x]);
    }
}

int oracle_hogbom_f32(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx,
                      double gain, double threshold, int64_t max_iter,
                      float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                      double *model, int64_t *n_iter_out, int32_t *stop_out)
{
    int st = check_common(ny, nx, psf_ny, psf_nx, gain, threshold, max_iter, comp_cap);
    if (st) return st;
    const int64_t npix = (int64_t)ny * nx;
    const float g = (float)gain;
    const int cy = psf_ny / 2, cx = psf_nx / 2;
    memmove(residual, dirty, sizeof(float) * npix);
    if (model) memset(model, 0, sizeof(double) * npix);
    int64_t n = 0;
    int32_t stop;
    for (;;) {
        /* find the highest-intensity pixel (Section 3, eq. 1) */
        int64_t p = peak_f32(residual, nx, 0, ny, 0, nx);
        float v = residual[p];
        if (n == max_iter) { stop = STOP_MAXITER; break; }
        if (!isfinite(v)) { stop = STOP_NONFINITE; break; }
        if ((double)fabsf(v) < threshold) { stop = STOP_THRESHOLD; break; }
        if (n == comp_cap) { stop = STOP_CAPACITY; break; }
        /* component = intensity x gain, saved with its position (eq. 1) */
        float c = g * v;
        comp_idx[n] = (int32_t)p;
        comp_flux[n] = c;
        if (model) model[p] += (double)c;
        /* residual -= intensity x gain x PSF at that position (eq. 2) */
        subtract_psf_f32(residual, nx, 0, ny, 0, nx, p, c, psf, psf_nx, cy, cx);
        n += 1;
    }
    *n_iter_out = n;
    *stop_out = stop;
    return OR_OK;
}

/* ---------------------------------------------------------------- FP64 -- */

/* The same order for doubles: magnitude bits, every NaN one value above +Inf. */
static uint64_t mag_f64(double v)
{
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    b &= 0x7FFFFFFFFFFFFFFFull;
    return b > 0x7FF0000000000000ull ? 0x7FF8000000000000ull : b;
}

static int64_t peak_f64(const double *r, int nx, int y0, int y1, int x0, int x1)
{
    uint64_t best = 0;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            uint64_t a = mag_f64(r[(int64_t)y * nx + x]);
            best = a > best ? a : best;
        }
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x)
            if (mag_f64(r[(int64_t)y * nx + x]) == best) return (int64_t)y * nx + x;
    return (int64_t)y0 * nx + x0;   /* not reached */
}

int64_t oracle_peak_f64(const double *r, int nx, int y0, int y1, int x0, int x1)
{
    if (nx <= 0 || y0 < 0 || x0 < 0 || y1 <= y0 || x1 <= x0 || x1 > nx) return -1;
    return peak_f64(r, nx, y0, y1, x0, x1);
}

static void subtract_psf_f64(double *r, int nx, int y0, int y1, int x0, int x1, int64_t p, double c,
                             const float *psf, int psf_nx, int cy, int cx)
{
    int py = (int)(p / nx), px = (int)(p % nx);
#pragma omp parallel for schedule(static) if ((int64_t)(y1 - y0) * (x1 - x0) > 65536)
    for (int y = y0; y < y1; ++y) {
        const float *prow = psf + (int64_t)(y - py + cy) * psf_nx + (cx - px);
        double *rrow = r + (int64_t)y * nx;
        for (int x = x0; x < x1; ++x)
            rrow[x] = fma(-c, (double)prow[x], rrow[x]);
    }
}

/* The same steps in double.  Inputs are the float32-stored dirty image and
 * PSF, promoted exactly, so a comparison with the FP32 run isolates the
 * arithmetic. */
int oracle_hogbom_f64(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx,
                      double gain, double threshold, int64_t max_iter,
                      double *residual, int32_t *comp_idx, double *comp_flux, int64_t comp_cap,
                      double *model, int64_t *n_iter_out, int32_t *stop_out)
{
    int st = check_common(ny, nx, psf_ny, psf_nx, gain, threshold, max_iter, comp_cap);
    if (st) return st;
    const int64_t npix = (int64_t)ny * nx;
    const int cy = psf_ny / 2, cx = psf_nx / 2;
    for (int64_t q = 0; q < npix; ++q) residual[q] = (double)dirty[q];
    if (model) memset(model, 0, sizeof(double) * npix);
    int64_t n = 0;
    int32_t stop;
    for (;;) {
        int64_t p = peak_f64(residual, nx, 0, ny, 0, nx);
        double v = residual[p];
        if (n == max_iter) { stop = STOP_MAXITER; break; }
        if (!isfinite(v)) { stop = STOP_NONFINITE; break; }
        if (fabs(v) < threshold) { stop = STOP_THRESHOLD; break; }
        if (n == comp_cap) { stop = STOP_CAPACITY; break; }
        double c = gain * v;
        comp_idx[n] = (int32_t)p;
        comp_flux[n] = c;
        if (model) model[p] += c;
        subtract_psf_f64(residual, nx, 0, ny, 0, nx, p, c, psf, psf_nx, cy, cx);
        n += 1;
    }
    *n_iter_out = n;
    *stop_out = stop;
    return OR_OK;
}

/* ------------------------------------------------------- tiled helpers -- */

typedef struct { int y0, y1, x0, x1; } rect;

static rect tile_rect(int ny, int nx, int ty, int tx, int t)
{
    int i = t / tx, j = t % tx;
    rect r;
    r.y0 = (int)((int64_t)i * ny / ty);
    r.y1 = (int)((int64_t)(i + 1) * ny / ty);
    r.x0 = (int)((int64_t)j * nx / tx);
    r.x1 = (int)((int64_t)(j + 1) * nx / tx);
    return r;
}

static int in_rect(rect r, int y, int x) { return y >= r.y0 && y < r.y1 && x >= r.x0 && x < r.x1; }

/* Per-round budgets: b_t = I when at least |A|*I iterations remain, else the
 * remainder R split evenly over the active tiles, the first (R mod |A|)
 * active tiles (in tile order) taking one more. */
static void round_budgets(const int *active, int ntiles, int64_t remaining, int interval, int64_t *budget)
{
    int64_t na = 0;
    for (int t = 0; t < ntiles; ++t) na += active[t];
    int64_t rank = 0;
    for (int t = 0; t < ntiles; ++t) {
        if (!active[t]) { budget[t] = 0; continue; }
        if (remaining >= na * (int64_t)interval) budget[t] = interval;
        else budget[t] = remaining / na + (rank < remaining % na ? 1 : 0);
        rank += 1;
    }
}

/* Cross-coupling feedback (Section 3, Fig. 2 and the text after it).
 * Component lists: entry k belongs to tile ctile[k], at flat index cidx[k],
 * with flux cflux[k]; entries are in the order they were found, and each lies
 * inside its own tile.
 *   1. Each tile's components are placed on a full-size component image: per
 *      pixel, the double sum of its components in list order, rounded once to
 *      the working precision.  The image is zero outside its own tile, so its
 *      non-zero pixels are collected by scanning that tile in raster order.
 *   2. For every pixel q, of tile s: the other tiles' cross-coupling images
 *      (component image convolved with the full PSF) are summed at q as one
 *      fma chain from zero, over tiles t != s in ascending order and each
 *      tile's non-zero pixels in raster order; then r[q] = r[q] - sum. */
typedef struct { int64_t n; int32_t *pos; } nzlist;

static int feedback_f32(float *r, int ny, int nx, int ty, int tx, const float *psf, int psf_nx, int cy, int cx,
                        const int32_t *ctile, const int32_t *cidx, const float *cflux, int64_t ncomp)
{
    const int64_t npix = (int64_t)ny * nx;
    const int ntiles = ty * tx;
    size_t m = (size_t)(ncomp > 0 ? ncomp : 1);
    double *cimg = (double *)calloc((size_t)npix, sizeof(double));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * m);
    float *val = (float *)malloc(sizeof(float) * m);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (ntiles + 1));
    if (!cimg || !pos || !val || !start) { free(cimg); free(pos); free(val); free(start); return OR_ENOMEM; }
    /* step 1: component images, as non-zero lists in raster order */
    for (int64_t k = 0; k < ncomp; ++k) cimg[cidx[k]] += (double)cflux[k];
    int64_t nnz = 0;
    for (int t = 0; t < ntiles; ++t) {
        rect own = tile_rect(ny, nx, ty, tx, t);
        start[t] = nnz;
        for (int y = own.y0; y < own.y1; ++y)
            for (int x = own.x0; x < own.x1; ++x) {
                int64_t q = (int64_t)y * nx + x;
                if (cimg[q] != 0.0) { pos[nnz] = (int32_t)q; val[nnz] = (float)cimg[q]; nnz++; }
            }
    }
    start[ntiles] = nnz;
    /* step 2: subtract the sum of the other tiles' cross-coupling images */
    for (int s = 0; s < ntiles; ++s) {
        rect own = tile_rect(ny, nx, ty, tx, s);
#pragma omp parallel for schedule(dynamic, 4) if (npix > 65536)
        for (int y = own.y0; y < own.y1; ++y)
            for (int x = own.x0; x < own.x1; ++x) {
                float acc = 0.0f;
                for (int t = 0; t < ntiles; ++t) {
                    if (t == s) continue;
                    for (int64_t j = start[t]; j < start[t + 1]; ++j) {
                        int py = pos[j] / nx, px = pos[j] % nx;
                        acc = fmaf(val[j], psf[(int64_t)(y - py + cy) * psf_nx + (x - px + cx)], acc);
                    }
                }
                r[(int64_t)y * nx + x] = r[(int64_t)y * nx + x] - acc;
            }
    }
    free(cimg); free(pos); free(val); free(start);
    return OR_OK;
}

static int feedback_f64(double *r, int ny, int nx, int ty, int tx, const float *psf, int psf_nx, int cy, int cx,
                        const int32_t *ctile, const int32_t *cidx, const double *cflux, int64_t ncomp)
{
    const int64_t npix = (int64_t)ny * nx;
    const int ntiles = ty * tx;
    size_t m = (size_t)(ncomp > 0 ? ncomp : 1);
    double *cimg = (double *)calloc((size_t)npix, sizeof(double));
    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * m);
    double *val = (double *)malloc(sizeof(double) * m);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (ntiles + 1));
    if (!cimg || !pos || !val || !start) { free(cimg); free(pos); free(val); free(start); return OR_ENOMEM; }
    for (int64_t k = 0; k < ncomp; ++k) cimg[cidx[k]] += cflux[k];
    int64_t nnz = 0;
    for (int t = 0; t < ntiles; ++t) {
        rect own = tile_rect(ny, nx, ty, tx, t);
        start[t] = nnz;
        for (int y = own.y0; y < own.y1; ++y)
            for (int x = own.x0; x < own.x1; ++x) {
                int64_t q = (int64_t)y * nx + x;
                if (cimg[q] != 0.0) { pos[nnz] = (int32_t)q; val[nnz] = cimg[q]; nnz++; }
            }
    }
    start[ntiles] = nnz;
    for (int s = 0; s < ntiles; ++s) {
        rect own = tile_rect(ny, nx, ty, tx, s);
#pragma omp parallel for schedule(dynamic, 4) if (npix > 65536)
        for (int y = own.y0; y < own.y1; ++y)
            for (int x = own.x0; x < own.x1; ++x) {
                double acc = 0.0;
                for (int t = 0; t < ntiles; ++t) {
                    if (t == s) continue;
                    for (int64_t j = start[t]; j < start[t + 1]; ++j) {
                        int py = pos[j] / nx, px = pos[j] % nx;
                        acc = fma(val[j], (double)psf[(int64_t)(y - py + cy) * psf_nx + (x - px + cx)], acc);
                    }
                }
                r[(int64_t)y * nx + x] -= acc;
            }
    }
    free(cimg); free(pos); free(val); free(start);
    return OR_OK;
}

static int lists_inside_tiles(int ny, int nx, int ty, int tx, const int32_t *ctile, const int32_t *cidx, int64_t ncomp)
{
    for (int64_t k = 0; k < ncomp; ++k) {
        if (ctile[k] < 0 || ctile[k] >= ty * tx || cidx[k] < 0 || (int64_t)cidx[k] >= (int64_t)ny * nx) return 0;
        rect tr = tile_rect(ny, nx, ty, tx, ctile[k]);
        if (!in_rect(tr, cidx[k] / nx, cidx[k] % nx)) return 0;
    }
    return 1;
}

/* Exposed for the feedback pin: applies one feedback step to r in place. */
int oracle_feedback_f32(float *r, int ny, int nx, int ty, int tx, const float *psf, int psf_ny, int psf_nx,
                        const int32_t *ctile, const int32_t *cidx, const float *cflux, int64_t ncomp)
{
    if (ny <= 0 || nx <= 0 || psf_ny < 2 * ny || psf_nx < 2 * nx || ty < 1 || tx < 1 || ty > ny || tx > nx)
        return OR_EINVAL;
    if (!lists_inside_tiles(ny, nx, ty, tx, ctile, cidx, ncomp)) return OR_EINVAL;
    return feedback_f32(r, ny, nx, ty, tx, psf, psf_nx, psf_ny / 2, psf_nx / 2, ctile, cidx, cflux, ncomp);
}

int oracle_feedback_f64(double *r, int ny, int nx, int ty, int tx, const float *psf, int psf_ny, int psf_nx,
                        const int32_t *ctile, const int32_t *cidx, const double *cflux, int64_t ncomp)
{
    if (ny <= 0 || nx <= 0 || psf_ny < 2 * ny || psf_nx < 2 * nx || ty < 1 || tx < 1 || ty > ny || tx > nx)
        return OR_EINVAL;
    if (!lists_inside_tiles(ny, nx, ty, tx, ctile, cidx, ncomp)) return OR_EINVAL;
    return feedback_f64(r, ny, nx, ty, tx, psf, psf_nx, psf_ny / 2, psf_nx / 2, ctile, cidx, cflux, ncomp);
}

/* ------------------------------------------------- tiled with feedback -- */

/* Tiled Hogbom CLEAN with feedback (Sections 2 and 3, Figs. 1-3), FP32.
 * Component output order: round, then tile, then local iteration. */
int oracle_tiled_f32(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx,
                     int tiles_y, int tiles_x, int interval, double level_frac,
                     double gain, double threshold, int64_t max_iter,
                     float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap,
                     double *model, int64_t *n_iter_out, int32_t *stop_out, int32_t *n_rounds_out)
{
    int st = check_common(ny, nx, psf_ny, psf_nx, gain, threshold, max_iter, comp_cap);
    if (st) return st;
    if (tiles_y < 1 || tiles_x < 1 || tiles_y > ny || tiles_x > nx || interval < 1) return OR_EINVAL;
    if (!(level_frac >= 0.0 && level_frac <= 1.0)) return OR_EINVAL;
    const int ntiles = tiles_y * tiles_x;
    const int64_t npix = (int64_t)ny * nx;
    const float g = (float)gain;
    const int cy = psf_ny / 2, cx = psf_nx / 2;
    memmove(residual, dirty, sizeof(float) * npix);
    if (model) memset(model, 0, sizeof(double) * npix);

    int *active = (int *)calloc(ntiles, sizeof(int));
    double *tpeak = (double *)calloc(ntiles, sizeof(double));
    int64_t *budget = (int64_t *)calloc(ntiles, sizeof(int64_t));
    int32_t *rtile = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntiles * interval);
    int32_t *ridx = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntiles * interval);
    float *rflux = (float *)malloc(sizeof(float) * (size_t)ntiles * interval);
    if (!active || !tpeak || !budget || !rtile || !ridx || !rflux) {
        free(active); free(tpeak); free(budget); free(rtile); free(ridx); free(rflux);
        return OR_ENOMEM;
    }
    const int64_t limit = max_iter < comp_cap ? max_iter : comp_cap;
    int64_t used = 0;
    int32_t rounds = 0, stop;
    for (;;) {
        /* each tile's current peak decides whether it takes part: at or above
         * the threshold, and at or above the round's flux level, the fraction
         * level_frac of the largest tile peak (0: every tile above threshold) */
        double vmax = 0.0;
        int nonfinite = 0;
        for (int t = 0; t < ntiles; ++t) {
            rect tr = tile_rect(ny, nx, tiles_y, tiles_x, t);
            tpeak[t] = (double)fabsf(residual[peak_f32(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1)]);
            nonfinite |= !isfinite(tpeak[t]);
            vmax = tpeak[t] > vmax ? tpeak[t] : vmax;
        }
        if (used == max_iter) { stop = STOP_MAXITER; break; }
        if (nonfinite) { stop = STOP_NONFINITE; break; }
        const double level = level_frac * vmax;
        int nactive = 0;
        for (int t = 0; t < ntiles; ++t) {
            active[t] = tpeak[t] >= threshold && tpeak[t] >= level;
            nactive += active[t];
        }
        if (nactive == 0) { stop = STOP_THRESHOLD; break; }
        if (used == comp_cap) { stop = STOP_CAPACITY; break; }
        round_budgets(active, ntiles, limit - used, interval, budget);

        /* every tile runs its own minor loop on its own pixels (Section 2) */
        int64_t nround = 0;
        for (int t = 0; t < ntiles; ++t) {
            rect tr = tile_rect(ny, nx, tiles_y, tiles_x, t);
            for (int64_t k = 0; k < budget[t]; ++k) {
                int64_t p = peak_f32(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1);
                float v = residual[p];
                if (!isfinite(v) || (double)fabsf(v) < threshold || (double)fabsf(v) < level) break;
                float c = g * v;
                rtile[nround] = t;
                ridx[nround] = (int32_t)p;
                rflux[nround] = c;
                nround++;
                subtract_psf_f32(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1, p, c, psf, psf_nx, cy, cx);
            }
        }
        for (int64_t k = 0; k < nround; ++k) {
            comp_idx[used + k] = ridx[k];
            comp_flux[used + k] = rflux[k];
            if (model) model[ridx[k]] += (double)rflux[k];
        }
        used += nround;
        rounds += 1;
        /* synchronising feedback step: cross-coupling of this round's
         * components subtracted from all other tiles (Section 3) */
        st = feedback_f32(residual, ny, nx, tiles_y, tiles_x, psf, psf_nx, cy, cx, rtile, ridx, rflux, nround);
        if (st) break;
    }
    free(active); free(tpeak); free(budget); free(rtile); free(ridx); free(rflux);
    if (st) return st;
    *n_iter_out = used;
    *stop_out = stop;
    *n_rounds_out = rounds;
    return OR_OK;
}

int oracle_tiled_f64(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx,
                     int tiles_y, int tiles_x, int interval, double level_frac,
                     double gain, double threshold, int64_t max_iter,
                     double *residual, int32_t *comp_idx, double *comp_flux, int64_t comp_cap,
                     double *model, int64_t *n_iter_out, int32_t *stop_out, int32_t *n_rounds_out)
{
    int st = check_common(ny, nx, psf_ny, psf_nx, gain, threshold, max_iter, comp_cap);
    if (st) return st;
    if (tiles_y < 1 || tiles_x < 1 || tiles_y > ny || tiles_x > nx || interval < 1) return OR_EINVAL;
    if (!(level_frac >= 0.0 && level_frac <= 1.0)) return OR_EINVAL;
    const int ntiles = tiles_y * tiles_x;
    const int64_t npix = (int64_t)ny * nx;
    const int cy = psf_ny / 2, cx = psf_nx / 2;
    for (int64_t q = 0; q < npix; ++q) residual[q] = (double)dirty[q];
    if (model) memset(model, 0, sizeof(double) * npix);

    int *active = (int *)calloc(ntiles, sizeof(int));
    double *tpeak = (double *)calloc(ntiles, sizeof(double));
    int64_t *budget = (int64_t *)calloc(ntiles, sizeof(int64_t));
    int32_t *rtile = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntiles * interval);
    int32_t *ridx = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntiles * interval);
    double *rflux = (double *)malloc(sizeof(double) * (size_t)ntiles * interval);
    if (!active || !tpeak || !budget || !rtile || !ridx || !rflux) {
        free(active); free(tpeak); free(budget); free(rtile); free(ridx); free(rflux);
        return OR_ENOMEM;
    }
    const int64_t limit = max_iter < comp_cap ? max_iter : comp_cap;
    int64_t used = 0;
    int32_t rounds = 0, stop;
    for (;;) {
        double vmax = 0.0;
        int nonfinite = 0;
        for (int t = 0; t < ntiles; ++t) {
            rect tr = tile_rect(ny, nx, tiles_y, tiles_x, t);
            tpeak[t] = fabs(residual[peak_f64(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1)]);
            nonfinite |= !isfinite(tpeak[t]);
            vmax = tpeak[t] > vmax ? tpeak[t] : vmax;
        }
        if (used == max_iter) { stop = STOP_MAXITER; break; }
        if (nonfinite) { stop = STOP_NONFINITE; break; }
        const double level = level_frac * vmax;
        int nactive = 0;
        for (int t = 0; t < ntiles; ++t) {
            active[t] = tpeak[t] >= threshold && tpeak[t] >= level;
            nactive += active[t];
        }
        if (nactive == 0) { stop = STOP_THRESHOLD; break; }
        if (used == comp_cap) { stop = STOP_CAPACITY; break; }
        round_budgets(active, ntiles, limit - used, interval, budget);
        int64_t nround = 0;
        for (int t = 0; t < ntiles; ++t) {
            rect tr = tile_rect(ny, nx, tiles_y, tiles_x, t);
            for (int64_t k = 0; k < budget[t]; ++k) {
                int64_t p = peak_f64(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1);
                double v = residual[p];
                if (!isfinite(v) || fabs(v) < threshold || fabs(v) < level) break;
                double c = gain * v;
                rtile[nround] = t;
                ridx[nround] = (int32_t)p;
                rflux[nround] = c;
                nround++;
                subtract_psf_f64(residual, nx, tr.y0, tr.y1, tr.x0, tr.x1, p, c, psf, psf_nx, cy, cx);
            }
        }
        for (int64_t k = 0; k < nround; ++k) {
            comp_idx[used + k] = ridx[k];
            comp_flux[used + k] = rflux[k];
            if (model) model[ridx[k]] += rflux[k];
        }
        used += nround;
        rounds += 1;
        st = feedback_f64(residual, ny, nx, tiles_y, tiles_x, psf, psf_nx, cy, cx, rtile, ridx, rflux, nround);
        if (st) break;
    }
    free(active); free(tpeak); free(budget); free(rtile); free(ridx); free(rflux);
    if (st) return st;
    *n_iter_out = used;
    *stop_out = stop;
    *n_rounds_out = rounds;
    return OR_OK;
}

/* ------------------------------------------------------- restoration -- */

/* The "reconstructed image" compared in Section 4 is not defined there; the
 * reading used here (and by the library) is the usual restored image: the
 * model convolved with a circular Gaussian clean beam of peak 1, plus the
 * residual.  The beam's FWHM is 2 sqrt(A / pi), with A the area in pixels of
 * the PSF's main lobe: the 4-connected region of values above one half that
 * contains the centre (psf_ny/2, psf_nx/2).  sigma = FWHM / (2 sqrt(2 ln 2)). */

/* Main-lobe area (pixels), by a breadth-first flood fill from the centre;
 * -1 if the centre is not above one half, -2 on allocation failure. */
int64_t oracle_main_lobe_area(const float *psf, int psf_ny, int psf_nx)
{
    if (psf_ny <= 0 || psf_nx <= 0) return -1;
    const int64_t n = (int64_t)psf_ny * psf_nx;
    const int64_t c = (int64_t)(psf_ny / 2) * psf_nx + psf_nx / 2;
    if (!(psf[c] > 0.5f)) return -1;
    unsigned char *seen = (unsigned char *)calloc((size_t)n, 1);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!seen || !queue) { free(seen); free(queue); return -2; }
    int64_t head = 0, tail = 0;
    queue[tail++] = c;
    seen[c] = 1;
    while (head < tail) {
        const int64_t q = queue[head++];
        const int y = (int)(q / psf_nx), x = (int)(q % psf_nx);
        const int ny4[4] = {y - 1, y + 1, y, y}, nx4[4] = {x, x, x - 1, x + 1};
        for (int k = 0; k < 4; ++k) {
            if (ny4[k] < 0 || ny4[k] >= psf_ny || nx4[k] < 0 || nx4[k] >= psf_nx) continue;
            const int64_t r = (int64_t)ny4[k] * psf_nx + nx4[k];
            if (!seen[r] && psf[r] > 0.5f) {
                seen[r] = 1;
                queue[tail++] = r;
            }
        }
    }
    free(seen);
    free(queue);
    return tail;
}

/* Restored image in float64: out[q] = residual[q] + sum over the square
 * window |dy|, |dx| <= R (R = ceil(5 sigma)) of model[q - d] * B(d), with
 * B(d) = exp(-(dy^2 + dx^2) / (2 sigma^2)) and pixels outside the image
 * counting as zero.  The sum runs in raster order of d. */
int oracle_restore_f64(const double *model, const float *residual, int ny, int nx, double sigma, double *out)
{
    if (ny <= 0 || nx <= 0 || !(sigma > 0.0) || sigma > 1000.0) return OR_EINVAL;
    const int R = (int)ceil(5.0 * sigma);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            double s = 0.0;
            for (int dy = -R; dy <= R; ++dy) {
                const int sy = y - dy;
                if (sy < 0 || sy >= ny) continue;
                for (int dx = -R; dx <= R; ++dx) {
                    const int sx = x - dx;
                    if (sx < 0 || sx >= nx) continue;
                    const double b = exp(-((double)dy * dy + (double)dx * dx) / (2.0 * sigma * sigma));
                    s += model[(int64_t)sy * nx + sx] * b;
                }
            }
            out[(int64_t)y * nx + x] = (double)residual[(int64_t)y * nx + x] + s;
        }
    }
    return OR_OK;
}
