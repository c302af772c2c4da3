// clean_fft.h -- transform primitives of the FFT form of the feedback step
// (the cross-coupling images of paper Section 3 computed as one circular
// convolution per round, for large images where the direct gather would read
// K_d * N^2 PSF values).
//
// Transforms run in LDS, one workgroup per transform or per block of short
// transforms, with twiddles W_L^m = exp(-2 pi i m / L) from a float table
// computed in double on the host:
//  * fft_lds / fft_lds_multi: iterative decimation in time, input placed in
//    bit-reversed order, stages two at a time;
//  * fft_big / fft13 (the wide-tile kernel): a padded LDS arena free of bank
//    conflicts, decimation in time or in frequency (no permutation pass for a
//    convolution), four stages per pass in registers, and at length 8192
//    compile-time LDS offsets and per-thread twiddles held in registers.
// Cross-workgroup buffers move through agent-coherent 8-byte loads and
// stores, or plain 8- and 16-byte ones between fenced grid barriers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clean_device.h"

namespace cleanhip {

// Agent-coherent 8-byte accesses: the FFT buffers are written by one
// workgroup and read by others within one launch.  Global address space, so
// that they count against the vector-memory counter only (a generic access
// also counts against the LDS one, and every LDS wait would wait for it).
typedef __attribute__((address_space(1))) const uint64_t gconst_u64;
typedef __attribute__((address_space(1))) uint64_t gmut_u64;
__device__ __forceinline__ float2 ldc2(const float2 *p)
{
    const uint64_t u = __hip_atomic_load((gconst_u64 *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
}
__device__ __forceinline__ void stc2(float2 *p, float2 v)
{
    const uint64_t u = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
    __hip_atomic_store((gmut_u64 *)p, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Plain 8- and 16-byte global accesses (no coherence bits, so they may stay
// in this XCD's L2): for buffers whose writers and readers a fenced grid
// barrier separates.  The 16-byte forms need a 16-byte aligned address.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f32x2 g_f32x2;
typedef __attribute__((address_space(1))) f32x4 g_f32x4;
__device__ __forceinline__ void stp2(float2 *p, float2 v) { *(g_f32x2 *)p = f32x2{v.x, v.y}; }
__device__ __forceinline__ void stp4(float2 *p, float2 u, float2 v) { *(g_f32x4 *)p = f32x4{u.x, u.y, v.x, v.y}; }
__device__ __forceinline__ float2 ldp2(const float2 *p)
{
    const f32x2 q = *(const g_f32x2 *)p;
    return make_float2(q.x, q.y);
}
__device__ __forceinline__ f32x4 ldp4(const float2 *p) { return *(const g_f32x4 *)p; }

// A workgroup-strided loop over e < n (e = threadIdx.x + m * WG) whose body
// reads global memory, then writes: the reads of U consecutive steps are
// issued before the first write, so U memory round trips overlap instead of
// following one another.  The reads are unconditional (indices past n read
// element n - 1 and are not written), since a branch between them would let
// the compiler wait for each read on its own; `load` must therefore return
// the raw values and leave every use to `put`.  With `sync`, a workgroup barrier separates the
// first reads from the first writes (for writes into LDS that other threads
// were reading before the call).  The loop bounds are uniform, so every
// thread reaches the barrier.
template <int U, class Load, class Put>
__device__ __forceinline__ void staged(int n, bool sync, Load load, Put put)
{
    using V = decltype(load(0));
    #pragma clang loop unroll(disable)
    for (int e0 = 0; e0 < n || (sync && e0 == 0); e0 += U * WG) {
        V v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)     // unconditional (index clamped): no branch between the loads
            v[u] = load(min(e0 + u * WG + (int)threadIdx.x, n - 1));
        if (sync && e0 == 0) __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * WG + (int)threadIdx.x;
            if (e < n) put(e, v[u]);
        }
    }
}

// LDS slot of element i of a transform: one spare slot after every 16
// elements and one more after every 256.  The passes read points at spacing
// 1 or 2 and the loaders write bit-reversed positions; unpadded, the 64 lanes
// of a wave would then hit one bank (addresses 32 B to 1 KB apart), padded
// they spread over all of them.  Every transform below works on padded
// segments; several segments of one pass lie fft_seg_stride(L) slots apart
// (odd, so that lanes running across segments also spread over the banks).
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4) + (i >> 8); }

__device__ __forceinline__ uint32_t bitrev(uint32_t i, int lg) { return __builtin_bitreverse32(i) >> (32 - lg); }

__device__ __forceinline__ float2 cmul(float2 p, float2 q)
{
    return make_float2(p.x * q.x - p.y * q.y, p.x * q.y + p.y * q.x);
}
__device__ __forceinline__ float2 cmulc(float2 p, float2 q)   // p * conj(q)
{
    return make_float2(p.x * q.x + p.y * q.y, p.y * q.x - p.x * q.y);
}

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

// radix4_unit with its flow graph transposed (stage s+1, then stage s).
__device__ __forceinline__ void radix4_unit_dif(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float2 w1, float2 w2,
                                                bool inverse)
{
    if (inverse) {
        w1.y = -w1.y;
        w2.y = -w2.y;
    }
    const float2 a0 = make_float2(x0.x + x2.x, x0.y + x2.y), a1 = make_float2(x1.x + x3.x, x1.y + x3.y);
    const float2 a2 = cmul(make_float2(x0.x - x2.x, x0.y - x2.y), w2);
    const float2 v = cmul(make_float2(x1.x - x3.x, x1.y - x3.y), w2);
    const float2 a3 = inverse ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
    x0 = make_float2(a0.x + a1.x, a0.y + a1.y);
    x1 = cmul(make_float2(a0.x - a1.x, a0.y - a1.y), w1);
    x2 = make_float2(a2.x + a3.x, a2.y + a3.y);
    x3 = cmul(make_float2(a2.x - a3.x, a2.y - a3.y), w1);
}

// `count` independent in-place transforms of length 2^lg, segment i at
// a[i * stride ..] (element e at slot pad16(e)), bit-reversed input, natural
// output; inverse: conjugate
// twiddles, no 1/L scaling.  tw is a table of W_L^m for a length
// L = 2^lg * tw_step (entries m < L/2 are read).  Stages go two at a time
// (radix 4: one thread reads four points, applies both radix-2 stages in
// registers and writes them back), after one plain radix-2 stage when lg is
// odd.  In a stage pair (s, s+1) the second stage's twiddle for the odd
// butterfly is W_4 times the even one's, an exact rotation by -i (+i for the
// inverse).  All threads of the workgroup.
__device__ inline void fft_lds_multi(float2 *a, int lg, int count, int stride, const float2 *tw, int tw_step,
                                     bool inverse)
{
    __syncthreads();
    int s = 0;
    if (lg & 1) {
        const int H = 1 << (lg - 1);
#pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * H; j += blockDim.x) {
            float2 *b = a + (j >> (lg - 1)) * stride + pad16(2 * (j & (H - 1)));   // 2j + 1 in the next slot
            const float2 u = b[0], v = b[1];
            b[0] = make_float2(u.x + v.x, u.y + v.y);
            b[1] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
        s = 1;
    }
    const int Q = lg >= 2 ? 1 << (lg - 2) : 0;
#pragma clang loop unroll(disable)
    for (; s < lg; s += 2) {
        const int half = 1 << s;
#pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * Q; j += blockDim.x) {
            const int jj = j & (Q - 1);
            const int k = jj & (half - 1);
            float2 *sg = a + (j >> (lg - 2)) * stride;
            const int e0 = ((jj >> s) << (s + 2)) + k;
            float2 *b0 = sg + pad16(e0), *b1 = sg + pad16(e0 + half), *b2 = sg + pad16(e0 + 2 * half),
                   *b3 = sg + pad16(e0 + 3 * half);
            float2 w1 = tw[(k << (lg - 1 - s)) * tw_step];
            float2 w2 = tw[(k << (lg - 2 - s)) * tw_step];
            if (inverse) {
                w1.y = -w1.y;
                w2.y = -w2.y;
            }
            const float2 x0 = *b0, x1 = *b1, x2 = *b2, x3 = *b3;
            const float2 p1 = cmul(x1, w1), p3 = cmul(x3, w1);
            const float2 a0 = make_float2(x0.x + p1.x, x0.y + p1.y), a1 = make_float2(x0.x - p1.x, x0.y - p1.y);
            const float2 a2 = make_float2(x2.x + p3.x, x2.y + p3.y), a3 = make_float2(x2.x - p3.x, x2.y - p3.y);
            const float2 t = cmul(a2, w2), v = cmul(a3, w2);
            const float2 u = inverse ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
            *b0 = make_float2(a0.x + t.x, a0.y + t.y);
            *b2 = make_float2(a0.x - t.x, a0.y - t.y);
            *b1 = make_float2(a1.x + u.x, a1.y + u.y);
            *b3 = make_float2(a1.x - u.x, a1.y - u.y);
        }
        __syncthreads();
    }
}

// fft_lds_multi in frequency order: natural input, bit-reversed output (its
// stages in reverse order, each butterfly transposed: radix4_unit_dif, then
// the plain radix-2 stage last when lg is odd).
__device__ inline void fft_lds_multi_dif(float2 *a, int lg, int count, int stride, const float2 *tw, int tw_step,
                                         bool inverse)
{
    __syncthreads();
    const int Q = lg >= 2 ? 1 << (lg - 2) : 0;
    #pragma clang loop unroll(disable)
    for (int s = lg - 2; s >= (lg & 1); s -= 2) {
        const int half = 1 << s;
        #pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * Q; j += blockDim.x) {
            const int jj = j & (Q - 1);
            const int k = jj & (half - 1);
            float2 *sg = a + (j >> (lg - 2)) * stride;
            const int e0 = ((jj >> s) << (s + 2)) + k;
            float2 *b0 = sg + pad16(e0), *b1 = sg + pad16(e0 + half), *b2 = sg + pad16(e0 + 2 * half),
                   *b3 = sg + pad16(e0 + 3 * half);
            float2 x0 = *b0, x1 = *b1, x2 = *b2, x3 = *b3;
            radix4_unit_dif(x0, x1, x2, x3, tw[(k << (lg - 1 - s)) * tw_step], tw[(k << (lg - 2 - s)) * tw_step],
                            inverse);
            *b0 = x0;
            *b1 = x1;
            *b2 = x2;
            *b3 = x3;
        }
        __syncthreads();
    }
    if (lg & 1) {
        const int H = 1 << (lg - 1);
        #pragma clang loop unroll(disable)
        for (int j = threadIdx.x; j < count * H; j += blockDim.x) {
            float2 *b = a + (j >> (lg - 1)) * stride + pad16(2 * (j & (H - 1)));
            const float2 u = b[0], v = b[1];
            b[0] = make_float2(u.x + v.x, u.y + v.y);
            b[1] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// In-place FFT of the padded arena a (length 2^lg; bit-reversed input,
// natural-order output), tw the table W_L^m of this length.  All threads of
// the workgroup.
__device__ inline void fft_lds(float2 *a, int lg, const float2 *tw, bool inverse)
{
    fft_lds_multi(a, lg, 1, fft_pad_slots(1 << lg), tw, 1, inverse);
}

// ------------------------------------------------------------------------
// Transforms of the wide-tile kernel (one workgroup per transform, length up
// to 8192, the workgroup's 512 threads holding up to 16 points each).
//
// Two orders: decimation in time (bit-reversed input, natural output, the
// passes of fft_lds_multi) and decimation in frequency (natural input,
// bit-reversed output).  The latter is the former's signal-flow graph
// transposed: the same stages in reverse order, each butterfly
// (u, v) -> (u + w v, u - w v) replaced by (a, b) -> (a + b, w (a - b)) with
// the same twiddle w.  A convolution along an axis then needs no permutation
// at all: forward in frequency order, product with a kernel spectrum held in
// the same (bit-reversed) order, inverse in time order.


// Stages s .. s+3 of a length-2^lg transform: a thread takes 16 points at
// spacing 2^s, both stage pairs in registers.
template <bool DIF>
__device__ __forceinline__ void big_pass16(float2 *a, int lg, int s, const float2 *tw, bool inverse)
{
    const int half = 1 << s, Q16 = 1 << (lg - 4);
    #pragma clang loop unroll(disable)
    for (int j = threadIdx.x; j < Q16; j += WG) {
        const int k = j & (half - 1);
        const int base = ((j >> s) << (s + 4)) + k;
        float2 x[16], w3[4], w4[4];
#pragma unroll
        for (int m = 0; m < 16; ++m) x[m] = a[pad16(base + m * half)];
        const float2 w1 = tw[k << (lg - 1 - s)], w2 = tw[k << (lg - 2 - s)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k2 = k + r * half;
            w3[r] = tw[k2 << (lg - 3 - s)];
            w4[r] = tw[k2 << (lg - 4 - s)];
        }
        if (!DIF) {
#pragma unroll
            for (int q = 0; q < 4; ++q) radix4_unit(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], w1, w2, inverse);
#pragma unroll
            for (int r = 0; r < 4; ++r) radix4_unit(x[r], x[r + 4], x[r + 8], x[r + 12], w3[r], w4[r], inverse);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) radix4_unit_dif(x[r], x[r + 4], x[r + 8], x[r + 12], w3[r], w4[r], inverse);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                radix4_unit_dif(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], w1, w2, inverse);
        }
#pragma unroll
        for (int m = 0; m < 16; ++m) a[pad16(base + m * half)] = x[m];
    }
    __syncthreads();
}

// Stages s, s+1: four points at spacing 2^s per unit.
template <bool DIF>
__device__ __forceinline__ void big_pass4(float2 *a, int lg, int s, const float2 *tw, bool inverse)
{
    const int half = 1 << s, Q = 1 << (lg - 2);
    #pragma clang loop unroll(disable)
    for (int j = threadIdx.x; j < Q; j += WG) {
        const int k = j & (half - 1);
        const int base = ((j >> s) << (s + 2)) + k;
        float2 x0 = a[pad16(base)], x1 = a[pad16(base + half)], x2 = a[pad16(base + 2 * half)],
               x3 = a[pad16(base + 3 * half)];
        const float2 w1 = tw[k << (lg - 1 - s)], w2 = tw[k << (lg - 2 - s)];
        if (!DIF) radix4_unit(x0, x1, x2, x3, w1, w2, inverse);
        else radix4_unit_dif(x0, x1, x2, x3, w1, w2, inverse);
        a[pad16(base)] = x0;
        a[pad16(base + half)] = x1;
        a[pad16(base + 2 * half)] = x2;
        a[pad16(base + 3 * half)] = x3;
    }
    __syncthreads();
}

// Stage 0 (twiddle 1; its own transpose).
__device__ __forceinline__ void big_pass2(float2 *a, int lg)
{
    #pragma clang loop unroll(disable)
    for (int j = threadIdx.x; j < (1 << (lg - 1)); j += WG) {
        const int i = pad16(2 * j);              // 2j + 1 sits in the next slot
        const float2 u = a[i], v = a[i + 1];
        a[i] = make_float2(u.x + v.x, u.y + v.y);
        a[i + 1] = make_float2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
}

// In-place transform of the padded arena a (length 2^lg, 2 <= lg <= 13), tw
// the table W_L^m of this length; inverse: conjugate twiddles, no scaling.
// DIF = false: bit-reversed input, natural output.  DIF = true: natural
// input, bit-reversed output.  All threads of the workgroup; starts and ends
// with a barrier.
template <bool DIF>
__device__ void fft_big(float2 *a, int lg, const float2 *tw, bool inverse)
{
    const int odd = lg & 1;
    const int n16 = (lg - odd) / 4;          // stages odd .. odd + 4 n16 - 1 in passes of four
    const int s4 = odd + 4 * n16;            // the rest in pairs
    __syncthreads();
    if (!DIF) {
        if (odd) big_pass2(a, lg);
        #pragma clang loop unroll(disable)
        for (int p = 0; p < n16; ++p) big_pass16<false>(a, lg, odd + 4 * p, tw, inverse);
        #pragma clang loop unroll(disable)
        for (int s = s4; s < lg; s += 2) big_pass4<false>(a, lg, s, tw, inverse);
    } else {
        #pragma clang loop unroll(disable)
        for (int s = lg - 2; s >= s4; s -= 2) big_pass4<true>(a, lg, s, tw, inverse);
        #pragma clang loop unroll(disable)
        for (int p = n16 - 1; p >= 0; --p) big_pass16<true>(a, lg, odd + 4 * p, tw, inverse);
        if (odd) big_pass2(a, lg);
    }
}

// ---- length 8192 (one workgroup of 512 threads, one 16-point unit per
// thread in every four-stage pass): the passes at stages 1-4, 5-8, 9-12 after
// (DIT) or before (DIF) stage 0.  Everything a thread touches is fixed by its
// index: its LDS slots are one base plus compile-time offsets, and its 30
// twiddles are loaded once per phase and kept in registers.

constexpr int F13 = 13;
__host__ __device__ constexpr int pad16c(int i) { return i + (i >> 4) + (i >> 8); }

// p * w, or p * conj(w) for the inverse, with fused multiply-adds.
template <bool INV> __device__ __forceinline__ float2 twmul(float2 p, float2 w)
{
    if (INV) return make_float2(fmaf(p.x, w.x, p.y * w.y), fmaf(p.y, w.x, -(p.x * w.y)));
    return make_float2(fmaf(p.x, w.x, -(p.y * w.y)), fmaf(p.x, w.y, p.y * w.x));
}

// radix4_unit (DIF = false) or radix4_unit_dif (DIF = true), the inverse a
// template argument.
template <bool DIF, bool INV>
__device__ __forceinline__ void unit4(float2 &x0, float2 &x1, float2 &x2, float2 &x3, float2 w1, float2 w2)
{
    auto add = [](float2 p, float2 q) { return make_float2(p.x + q.x, p.y + q.y); };
    auto sub = [](float2 p, float2 q) { return make_float2(p.x - q.x, p.y - q.y); };
    auto rot = [](float2 v) { return INV ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x); };   // * -+i
    if (!DIF) {
        const float2 p1 = twmul<INV>(x1, w1), p3 = twmul<INV>(x3, w1);
        const float2 a0 = add(x0, p1), a1 = sub(x0, p1), a2 = add(x2, p3), a3 = sub(x2, p3);
        const float2 t = twmul<INV>(a2, w2), u = rot(twmul<INV>(a3, w2));
        x0 = add(a0, t);
        x2 = sub(a0, t);
        x1 = add(a1, u);
        x3 = sub(a1, u);
    } else {
        const float2 a0 = add(x0, x2), a1 = add(x1, x3);
        const float2 a2 = twmul<INV>(sub(x0, x2), w2), a3 = rot(twmul<INV>(sub(x1, x3), w2));
        x0 = add(a0, a1);
        x1 = twmul<INV>(sub(a0, a1), w1);
        x2 = add(a2, a3);
        x3 = twmul<INV>(sub(a2, a3), w1);
    }
}

// The thread's twiddles of the three four-stage passes (S = 1, 5, 9):
// w1, w2 of stages S, S+1 and w3[r], w4[r] of stages S+2, S+3 for the four
// groups r, from the table W_L^m (m < L/2).
struct Tw13 {
    float2 w[3][10];
};
__device__ __forceinline__ void tw13_load(Tw13 &T, const float2 *tw)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int S = 1 + 4 * p, half = 1 << S, k = t & (half - 1);
        T.w[p][0] = tw[k << (F13 - 1 - S)];
        T.w[p][1] = tw[k << (F13 - 2 - S)];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T.w[p][2 + r] = tw[(k + r * half) << (F13 - 3 - S)];
            T.w[p][6 + r] = tw[(k + r * half) << (F13 - 4 - S)];
        }
    }
}

// Stages S .. S+3; the unit's 16 slots are pad16(base) plus offsets that do
// not depend on the thread (for these S the padding of base + m * 2^S splits
// into the padding of base and of m * 2^S).
template <int S, bool DIF, bool INV>
__device__ __forceinline__ void f13_units(float2 (&x)[16], const float2 (&w)[10])
{
    if (!DIF) {
#pragma unroll
        for (int q = 0; q < 4; ++q) unit4<false, INV>(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], w[0], w[1]);
#pragma unroll
        for (int r = 0; r < 4; ++r) unit4<false, INV>(x[r], x[r + 4], x[r + 8], x[r + 12], w[2 + r], w[6 + r]);
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) unit4<true, INV>(x[r], x[r + 4], x[r + 8], x[r + 12], w[2 + r], w[6 + r]);
#pragma unroll
        for (int q = 0; q < 4; ++q) unit4<true, INV>(x[4 * q], x[4 * q + 1], x[4 * q + 2], x[4 * q + 3], w[0], w[1]);
    }
}

// The thread's first slot in the pass at stages S .. S+3.  At S = 9 the
// unit's 16 points are elements t + 512 m, the thread's natural-order
// elements, so that pass can take its input from registers (frequency order)
// or leave its output there (time order).
template <int S> __device__ __forceinline__ float2 *f13_base(float2 *a)
{
    const int t = threadIdx.x;
    return a + pad16(((t >> S) << (S + 4)) + (t & ((1 << S) - 1)));
}

template <int S, bool DIF, bool INV>
__device__ __forceinline__ void f13_pass16(float2 *a, const float2 (&w)[10])
{
    constexpr int half = 1 << S;
    float2 *b = f13_base<S>(a);
    float2 x[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) x[m] = b[pad16c(m * half)];
    f13_units<S, DIF, INV>(x, w);
#pragma unroll
    for (int m = 0; m < 16; ++m) b[pad16c(m * half)] = x[m];
    __syncthreads();
}

// Stage 0: pairs (2j, 2j+1), j = t + 512 m.
__device__ __forceinline__ void f13_pass2(float2 *a)
{
    float2 *b = a + pad16(2 * (int)threadIdx.x);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int o = pad16c(1024 * m);
        const float2 u = b[o], v = b[o + 1];
        b[o] = make_float2(u.x + v.x, u.y + v.y);
        b[o + 1] = make_float2(u.x - v.x, u.y - v.y);
    }
    __syncthreads();
}

// The length-8192 transform of the padded arena; DIF / DIT as fft_big.
template <bool DIF, bool INV>
__device__ __forceinline__ void fft13(float2 *a, const Tw13 &T)
{
    __syncthreads();
    if (!DIF) {
        f13_pass2(a);
        f13_pass16<1, false, INV>(a, T.w[0]);
        f13_pass16<5, false, INV>(a, T.w[1]);
        f13_pass16<9, false, INV>(a, T.w[2]);
    } else {
        f13_pass16<9, true, INV>(a, T.w[2]);
        f13_pass16<5, true, INV>(a, T.w[1]);
        f13_pass16<1, true, INV>(a, T.w[0]);
        f13_pass2(a);
    }
}

// Puts a natural-order padded arena into bit-reversed order, in place.
__device__ inline void bitrev_permute(float2 *a, int lg)
{
    __syncthreads();
    const int L = 1 << lg;
    #pragma clang loop unroll(disable)
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const int j = (int)bitrev((uint32_t)i, lg);
        if (i < j) {
            const float2 t = a[pad16(i)];
            a[pad16(i)] = a[pad16(j)];
            a[pad16(j)] = t;
        }
    }
    __syncthreads();
}

} // namespace cleanhip
