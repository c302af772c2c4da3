// clean_restore.hip -- kernels of the restored image: the model convolved
// with a circular Gaussian clean beam of peak 1, plus the residual (the usual
// reading of the reconstructed image the paper compares in Section 4).
//
// Restored = model (*) B + residual, B(d) = b(dy) b(dx) with
// b(t) = exp(-t^2 / (2 sigma^2)), |t| <= R: separable, so two passes of
// 2R + 1 taps (rows, then columns) in float64.  One thread per output pixel;
// neighbouring threads share their taps through L1.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cleanhip {

__global__ void __launch_bounds__(256) restore_rows_kernel(const double *model, double *tmp, int ny, int nx,
                                                           const double *b, int R)
{
    const int64_t n = (int64_t)ny * nx;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / nx), x = (int)(i % nx);
        const int lo = max(-R, x - nx + 1), hi = min(R, x);      // source column x - d inside the image
        const double *row = model + (int64_t)y * nx;
        double s = 0.0;
        for (int d = lo; d <= hi; ++d) s = __builtin_fma(row[x - d], b[d + R], s);
        tmp[i] = s;
    }
}

__global__ void __launch_bounds__(256) restore_cols_kernel(const double *tmp, const float *residual, double *out,
                                                           int ny, int nx, const double *b, int R)
{
    const int64_t n = (int64_t)ny * nx;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / nx), x = (int)(i % nx);
        const int lo = max(-R, y - ny + 1), hi = min(R, y);
        double s = 0.0;
        for (int d = lo; d <= hi; ++d) s = __builtin_fma(tmp[(int64_t)(y - d) * nx + x], b[d + R], s);
        out[i] = (double)residual[i] + s;
    }
}

// Per block: the smallest and largest a[i] - b[i] of its grid-stride share
// (NaN in both when any difference is NaN), to part[2 * block], part[2 * block + 1].
__global__ void __launch_bounds__(256) diff_range_kernel(const double *a, const double *b, int64_t n, double *part)
{
    __shared__ double s_lo[256], s_hi[256];
    double lo = INFINITY, hi = -INFINITY;
    bool nan = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = a[i] - b[i];
        nan = nan || d != d;
        lo = fmin(lo, d);
        hi = fmax(hi, d);
    }
    s_lo[threadIdx.x] = nan ? NAN : lo;
    s_hi[threadIdx.x] = nan ? NAN : hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        double l = s_lo[0], h = s_hi[0];
        for (int t = 1; t < 256; ++t) {
            if (s_lo[t] != s_lo[t] || l != l) { l = NAN; h = NAN; continue; }
            l = fmin(l, s_lo[t]);
            h = fmax(h, s_hi[t]);
        }
        part[2 * blockIdx.x] = l;
        part[2 * blockIdx.x + 1] = h;
    }
}

} // namespace cleanhip
