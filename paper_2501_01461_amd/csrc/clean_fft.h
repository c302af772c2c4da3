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

__device__ __forceinline__ float2 cmul(float2 p, float2 q)
{
    return make_float2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x);
}
__device__ __forceinline__ float2 cmulc(float2 p, float2 q)   // p * conj(q)
{
    return make_float2(p.x * q.x + p.y * q.y, p.y * q.x - p.x * q.y);
}

// `count` independent in-place transforms of length 2^lg, segment i at
// a[i * stride ..], bit-reversed input, natural output; inverse: conjugate
// twiddles, no 1/L scaling.  tw is a table of W_L^m for a length
// L = 2^lg * tw_step (entries m < L/2 are read).  Stages go two at a time
// (radix 4: one thread reads four points, applies both radix-2 stages in
// registers and writes them back), after one plain radix-2 stage when lg is
// odd.  In a stage pair (s, s+1) the second stage's twiddle for the odd
// butterfly is W_4 times the even one's, an exact rotation by -i (+i for the
// inverse).  All threads of the workgroup.
// One radix-4 unit: stage pair (s, s+1) on x0..x3 at spacing 2^s, twiddles w1
// (stage s) and w2 (stage s+1); the arithmetic of fft_lds_multi's passes.
__device__ __forceinline__ void radix4_unit(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float2 w1, float2 w2,
                                            bool inverse)
{
    if (inverse) {
        w1.y = -w1.y;
        w2.y = -w2.y;
    }
    const float2 p1 = cmul(x1, w1), p3 = cmul(x3, w1);
    const float2 a0 = make_float2(x0.x + p1.x, x0.y + p1.y), a1 = make_float2(x0.x - p1.x, x0.y - p1.y);
    const float2 a2 = make_float2(x2.x + p3.x, x2.y + p3.y), a3 = make_float2(x2.x - p3.x, x2.y - p3.y);
    const float2 t = cmul(a2, w2), v = cmul(a3, w2);
    const float2 u = inverse ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
    x0 = make_float2(a0.x + t.x, a0.y + t.y);
    x2 = make_float2(a0.x - t.x, a0.y - t.y);
    x1 = make_float2(a1.x + u.x, a1.y + u.y);
    x3 = make_float2(a1.x - u.x, a1.y - u.y);
}

// R16: while four stages remain, a thread takes 16 points at spacing 2^s and
// applies both stage pairs (s, s+1) and (s+2, s+3) in registers, as four
// radix-4 units each: the same operations on the same values as two radix-4
// passes (bit-identical), with one LDS round trip and one barrier instead of
// two.  Needs the registers of 16 points; used where the kernel has them.
template <bool R16 = false>
__device__ inline void fft_lds_multi(float2 *a, int lg, int count, int stride, const float2 *tw, int tw_step,
                                     bool inverse)
{
    __syncthreads();
    int s = 0;
    if (lg & 1) {
        const int H = 1 << (lg - 1);
#pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * H; j += blockDim.x) {
            float2 *b = a + (j >> (lg - 1)) * stride + 2 * (j & (H - 1));
            const float2 u = b[0], v = b[1];
            b[0] = make_float2(u.x + v.x, u.y + v.y);
            b[1] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
        s = 1;
    }
    if constexpr (R16) {
        const int Q16 = lg >= 4 ? 1 << (lg - 4) : 0;
#pragma clang loop unroll(disable)
        for (; s + 4 <= lg; s += 4) {
            const int half = 1 << s;
#pragma clang loop unroll(disable)
            for (int j = threadIdx.x; j < count * Q16; j += blockDim.x) {
                const int jj = j & (Q16 - 1);
                const int k = jj & (half - 1);
                float2 *b = a + (j >> (lg - 4)) * stride + ((jj >> s) << (s + 4)) + k;
                float2 x[16];
#pragma unroll
                for (int m = 0; m < 16; ++m) x[m] = b[m * half];
                const float2 w1 = tw[(k << (lg - 1 - s)) * tw_step], w2 = tw[(k << (lg - 2 - s)) * tw_step];
#pragma unroll
                for (int q = 0; q < 4; ++q) radix4_unit(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], w1, w2, inverse);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k2 = k + r * half;
                    radix4_unit(x[r], x[r + 4], x[r + 8], x[r + 12], tw[(k2 << (lg - 3 - s)) * tw_step],
                                tw[(k2 << (lg - 4 - s)) * tw_step], inverse);
                }
#pragma unroll
                for (int m = 0; m < 16; ++m) b[m * half] = x[m];
            }
            __syncthreads();
        }
    }
    const int Q = lg >= 2 ? 1 << (lg - 2) : 0;
#pragma clang loop unroll(disable)
    for (; s < lg; s += 2) {
        const int half = 1 << s;
#pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * Q; j += blockDim.x) {
            const int jj = j & (Q - 1);
            const int k = jj & (half - 1);
            float2 *b = a + (j >> (lg - 2)) * stride + ((jj >> s) << (s + 2)) + k;
            float2 w1 = tw[(k << (lg - 1 - s)) * tw_step];
            float2 w2 = tw[(k << (lg - 2 - s)) * tw_step];
            if (inverse) {
                w1.y = -w1.y;
                w2.y = -w2.y;
            }
            const float2 x0 = b[0], x1 = b[half], x2 = b[2 * half], x3 = b[3 * half];
            const float2 p1 = cmul(x1, w1), p3 = cmul(x3, w1);
            const float2 a0 = make_float2(x0.x + p1.x, x0.y + p1.y), a1 = make_float2(x0.x - p1.x, x0.y - p1.y);
            const float2 a2 = make_float2(x2.x + p3.x, x2.y + p3.y), a3 = make_float2(x2.x - p3.x, x2.y - p3.y);
            const float2 t = cmul(a2, w2), v = cmul(a3, w2);
            const float2 u = inverse ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
            b[0] = make_float2(a0.x + t.x, a0.y + t.y);
            b[2 * half] = make_float2(a0.x - t.x, a0.y - t.y);
            b[half] = make_float2(a1.x + u.x, a1.y + u.y);
            b[3 * half] = make_float2(a1.x - u.x, a1.y - u.y);
        }
        __syncthreads();
    }
}

// In-place FFT of a[0 .. 2^lg) (bit-reversed input, natural-order output),
// tw the table W_L^m of this length.  All threads of the workgroup.
template <bool R16 = false>
__device__ inline void fft_lds(float2 *a, int lg, const float2 *tw, bool inverse)
{
    fft_lds_multi<R16>(a, lg, 1, 1 << lg, tw, 1, inverse);
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
//
// G > 1: the workgroup takes G tiles at a time (lds holds G tiles) and a
// thread issues its loads of all of them before the first LDS write, so one
// memory round trip serves G tiles.  Needs the registers of 2G values.
template <int G = 1>
__device__ inline void transpose_tiles(const float2 *src, int ss, float2 *dst, int ds, int rows, int cols, int w0,
                                       int nwork, float2 (*lds)[33])
{
    if constexpr (G > 1) {
        constexpr int PER = 1024 / WG;   // elements of one tile per thread
        const int tr = (rows + 31) / 32, tc = (cols + 31) / 32, nt = tr * tc;
        #pragma clang loop unroll(disable)
        for (int t0 = w0; t0 < nt; t0 += G * nwork) {
            float2 v[G][PER] = {};
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = t0 + g * nwork;
                const int br = (t / tc) * 32, bc = (t % tc) * 32;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int e = (int)threadIdx.x + k * WG, r = e / 32, c = e % 32;
                    if (t < nt && br + r < rows && bc + c < cols) v[g][k] = ldc2(&src[(size_t)(br + r) * ss + bc + c]);
                }
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int e = (int)threadIdx.x + k * WG;
                    lds[g * 32 + e / 32][e % 32] = v[g][k];
                }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int t = t0 + g * nwork;
                const int br = (t / tc) * 32, bc = (t % tc) * 32;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int e = (int)threadIdx.x + k * WG, c = e / 32, r = e % 32;
                    if (t < nt && br + r < rows && bc + c < cols)
                        stc2(&dst[(size_t)(bc + c) * ds + br + r], lds[g * 32 + r][c]);
                }
            }
        }
        return;
    }
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
