/* The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: plain
 * and tiled runs (FP32 and FP64) on small ragged images, with every stop
 * rule, the flux trigger, tiny tiles and capacity limits, the feedback step
 * on its own, the main-lobe area and the restoration, and argument errors.
 * Exit status 0 when no sanitizer fires and every call returns as expected. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t oracle_peak_f32(const float *r, int nx, int y0, int y1, int x0, int x1);
int oracle_hogbom_f32(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx, double gain,
                      double threshold, int64_t max_iter, float *residual, int32_t *comp_idx, float *comp_flux,
                      int64_t comp_cap, double *model, int64_t *n_iter_out, int32_t *stop_out);
int oracle_hogbom_f64(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx, double gain,
                      double threshold, int64_t max_iter, double *residual, int32_t *comp_idx, double *comp_flux,
                      int64_t comp_cap, double *model, int64_t *n_iter_out, int32_t *stop_out);
int oracle_tiled_f32(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx, int tiles_y,
                     int tiles_x, int interval, double level_frac, double gain, double threshold, int64_t max_iter,
                     float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap, double *model,
                     int64_t *n_iter_out, int32_t *stop_out, int32_t *n_rounds_out);
int oracle_tiled_f64(const float *dirty, int ny, int nx, const float *psf, int psf_ny, int psf_nx, int tiles_y,
                     int tiles_x, int interval, double level_frac, double gain, double threshold, int64_t max_iter,
                     double *residual, int32_t *comp_idx, double *comp_flux, int64_t comp_cap, double *model,
                     int64_t *n_iter_out, int32_t *stop_out, int32_t *n_rounds_out);
int64_t oracle_main_lobe_area(const float *psf, int psf_ny, int psf_nx);
int oracle_restore_f64(const double *model, const float *residual, int ny, int nx, double sigma, double *out);

static int failures = 0;
#define EXPECT(c)                                                         \
    do {                                                                  \
        if (!(c)) {                                                       \
            fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #c);        \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static uint64_t state = 88172645463325252ull;
static double uni(void)    /* xorshift64, [0, 1) */
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

int main(void)
{
    const int shapes[][2] = {{1, 1}, {1, 9}, {7, 3}, {17, 23}, {32, 32}, {45, 64}};
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
        const int ny = shapes[s][0], nx = shapes[s][1], py = 2 * ny + (int)(s % 2), px = 2 * nx + 2;
        const int64_t npix = (int64_t)ny * nx, cap = 300;
        float *dirty = malloc(sizeof(float) * npix), *psf = malloc(sizeof(float) * py * px);
        float *res = malloc(sizeof(float) * npix), *flux = malloc(sizeof(float) * cap);
        double *res64 = malloc(sizeof(double) * npix), *flux64 = malloc(sizeof(double) * cap);
        double *model = malloc(sizeof(double) * npix), *rest = malloc(sizeof(double) * npix);
        int32_t *idx = malloc(sizeof(int32_t) * cap);
        for (int64_t i = 0; i < npix; ++i) dirty[i] = (float)(uni() < 0.1 ? 4.0 * uni() - 2.0 : 0.02 * (uni() - 0.5));
        for (int i = 0; i < py * px; ++i) psf[i] = (float)(0.6 * uni() - 0.3);
        psf[(py / 2) * px + px / 2] = 1.0f;
        int64_t n = 0;
        int32_t stop = -1, rounds = 0;
        EXPECT(oracle_peak_f32(dirty, nx, 0, ny, 0, nx) >= 0);
        for (int t = 0; t < 3; ++t) {
            const double thr = t == 1 ? 0.5 : 0.0;
            const int64_t c = t == 2 ? 5 : cap;
            EXPECT(oracle_hogbom_f32(dirty, ny, nx, psf, py, px, 0.1, thr, 200, res, idx, flux, c, model, &n, &stop) == 0);
            EXPECT(n <= 200 && n <= c);
            EXPECT(oracle_hogbom_f64(dirty, ny, nx, psf, py, px, 0.1, thr, 200, res64, idx, flux64, c, model, &n,
                                     &stop) == 0);
            const int ty = ny >= 3 ? 3 : ny, tx = nx >= 2 ? 2 : nx;
            EXPECT(oracle_tiled_f32(dirty, ny, nx, psf, py, px, ty, tx, 7, t == 0 ? 0.0 : 0.5, 0.1, thr, 200, res,
                                    idx, flux, c, model, &n, &stop, &rounds) == 0);
            EXPECT(oracle_tiled_f64(dirty, ny, nx, psf, py, px, ty, tx, 7, 0.0, 0.1, thr, 200, res64, idx, flux64, c,
                                    model, &n, &stop, &rounds) == 0);
            EXPECT(oracle_tiled_f32(dirty, ny, nx, psf, py, px, ny, nx, 3, 0.0, 0.1, thr, 100, res, idx, flux, c,
                                    model, &n, &stop, &rounds) == 0);   /* one-pixel tiles */
        }
        EXPECT(oracle_main_lobe_area(psf, py, px) >= 1);
        EXPECT(oracle_restore_f64(model, res, ny, nx, 1.7, rest) == 0);
        EXPECT(oracle_restore_f64(model, res, ny, nx, 0.0, rest) != 0);
        /* argument errors */
        EXPECT(oracle_hogbom_f32(dirty, ny, nx, psf, py - 2, px, 0.1, 0.0, 10, res, idx, flux, cap, model, &n, &stop) != 0);
        EXPECT(oracle_tiled_f32(dirty, ny, nx, psf, py, px, ny + 1, 1, 7, 0.0, 0.1, 0.0, 10, res, idx, flux, cap, model,
                                &n, &stop, &rounds) != 0);
        free(dirty); free(psf); free(res); free(flux); free(res64); free(flux64); free(model); free(rest); free(idx);
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle driver: all checks passed\n");
    return 0;
}
