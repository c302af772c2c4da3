// clean_fft.h -- transform primitives of the FFT form of the feedback step
// (the cross-coupling images of paper Section 3 computed as one circular
// convolution per round, for large images where the direct gather would read
// K_d * N^2 PSF values).
//
// Transforms run in LDS, one workgroup per transform or per block of short
// transforms: iterative radix-2 decimation in time, input placed in
// bit-reversed order, twiddles W_L^m = exp(-2 pi i m / L) from a float table
// computed in double on the host.  Cross-workgroup buffers move through
// agent-coherent 8-byte loads and stores; transposes through 32 x 33 LDS tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clean_device.h"

namespace cleanhip {

// Agent-coherent 8-byte accesses: the FFT buffers are written by one
// workgroup and read by others within one launch.
__device__ __forceinline__ float2 ldc2(const float2 *p)
{
    const uint64_t u = __hip_atomic_load((const uint64_t *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
}
__device__ __forceinline__ void stc2(float2 *p, float2 v)
{
    const uint64_t u = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
    __hip_atomic_store((uint64_t *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t bitrev(uint32_t i, int lg) { return __builtin_bitreverse32(i) >> (32 - lg); }

// In-place FFT of a[0 .. 2^lg) (bit-reversed input, natural-order output).
// inverse: conjugate twiddles (no 1/L scaling).  All threads of the workgroup.
__device__ inline void fft_lds(float2 *a, int lg, const float2 *tw, bool inverse)
{
    const int H = 1 << (lg - 1);
    __syncthreads();
    #pragma clang loop unroll(disable)
    for (int s = 0; s < lg; ++s) {
        const int half = 1 << s;
        #pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < H; j += blockDim.x) {
            const int k = j & (half - 1);
            const int i0 = ((j >> s) << (s + 1)) + k, i1 = i0 + half;
            float2 w = tw[k << (lg - 1 - s)];
            if (inverse) w.y = -w.y;
            const float2 u = a[i0], v = a[i1];
            const float2 t = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
            a[i0] = make_float2(u.x + t.x, u.y + t.y);
            a[i1] = make_float2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
}

// `count` independent in-place transforms of length 2^lg, segment i at
// a[i * stride ..], bit-reversed input, natural output.  tw is a table of
// W_L^m for a length L = 2^lg * tw_step (entries m < L/2 are read).
__device__ inline void fft_lds_multi(float2 *a, int lg, int count, int stride, const float2 *tw, int tw_step,
                                     bool inverse)
{
    const int H = 1 << (lg - 1);
    const int total = count * H;
    __syncthreads();
    #pragma clang loop unroll(disable)
    for (int s = 0; s < lg; ++s) {
        const int half = 1 << s;
        #pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < total; j += blockDim.x) {
            const int seg = j >> (lg - 1), jj = j & (H - 1);
            const int k = jj & (half - 1);
            float2 *b = a + seg * stride;
            const int i0 = ((jj >> s) << (s + 1)) + k, i1 = i0 + half;
            float2 w = tw[(k << (lg - 1 - s)) * tw_step];
            if (inverse) w.y = -w.y;
            const float2 u = b[i0], v = b[i1];
            const float2 t = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
            b[i0] = make_float2(u.x + t.x, u.y + t.y);
            b[i1] = make_float2(u.x - t.x, u.y - t.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ float2 cmul(float2 p, float2 q)
{
    return make_float2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x);
}
__device__ __forceinline__ float2 cmulc(float2 p, float2 q)   // p * conj(q)
{
    return make_float2(p.x * q.x + p.y * q.y, p.y * q.x - p.x * q.y);
}

// Puts a natural-order array into bit-reversed order, in place.
__device__ inline void bitrev_permute(float2 *a, int lg)
{
    __syncthreads();
    const int L = 1 << lg;
    #pragma clang loop unroll(disable)
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const int j = (int)bitrev((uint32_t)i, lg);
        if (i < j) {
            const float2 t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    __syncthreads();
}

// 32 x 32 tiled transpose of the rows [0, rows) x columns [0, cols) of `src`
// (row stride ss) into dst (row stride ds): dst[c][r] = src[r][c].  Tiles are
// dealt over the workgroups (work item w of nwork).
__device__ inline void transpose_tiles(const float2 *src, int ss, float2 *dst, int ds, int rows, int cols, int w0,
                                       int nwork, float2 (*lds)[33])
{
    const int tr = (rows + 31) / 32, tc = (cols + 31) / 32;
    #pragma clang loop unroll(disable)
    for (int t = w0; t < tr * tc; t += nwork) {
        const int br = (t / tc) * 32, bc = (t % tc) * 32;
        __syncthreads();
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
            const int r = e / 32, c = e % 32;
            if (br + r < rows && bc + c < cols) lds[r][c] = ldc2(&src[(size_t)(br + r) * ss + bc + c]);
        }
        __syncthreads();
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
            const int c = e / 32, r = e % 32;
            if (br + r < rows && bc + c < cols) stc2(&dst[(size_t)(bc + c) * ds + br + r], lds[r][c]);
        }
    }
}

} // namespace cleanhip
