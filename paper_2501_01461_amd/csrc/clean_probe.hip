// clean_probe.hip -- memory-bandwidth probes that give the roofline
// denominators of the CLEAN kernels on the device they run on: the read
// bandwidth a working set of a given size achieves (L2-, Infinity-Cache- or
// HBM-resident, depending on its size), and the copy bandwidth.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cleanhip {

// Every thread reads 16-byte words in a grid-stride loop over the buffer,
// `reps` times; the same workgroup reads the same words each time, so a
// working set small enough for the caches is served from them after the
// first pass.  The sum keeps the loads alive (written only if it is an
// impossible value).
__global__ void __launch_bounds__(256) probe_read_kernel(const float4 *p, int64_t n4, int reps, float *sink)
{
    float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < reps; ++r) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += 4 * stride) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = i + u * stride;
                v[u] = j < n4 ? p[j] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ax += v[u].x; ay += v[u].y; az += v[u].z; aw += v[u].w;
            }
        }
    }
    if (ax + ay + az + aw == -1.2345e-30f) sink[threadIdx.x] = ax;
}

// dst[i] = src[i], 16-byte words, grid-stride.
__global__ void __launch_bounds__(256) probe_copy_kernel(const float4 *src, float4 *dst, int64_t n4, int reps)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < reps; ++r)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

} // namespace cleanhip
