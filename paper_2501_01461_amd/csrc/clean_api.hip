// clean_api.hip -- host entry points of the CLEAN library (the C ABI declared
// in include/clean.h): argument checks, workspace, launch shape, workgroup
// placement over the XCDs, cooperative launch, statistics.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "clean.h"
#include "clean_device.h"

namespace cleanhip {
template <int K, int V, typename PT> struct RegTile;
template <int K, int V, typename PT> struct StreamTile;
template <typename PT> struct WideTile;
template <class Tile> __global__ void hogbom_kernel(const KArgs a);
template <class Tile, bool FFT> __global__ void tiled_kernel(const KArgs a);
template <class Tile, bool TILED> __global__ void batched_kernel(const BatchArgs b);
__global__ void finalize_batch_kernel(const PlainJob *jobs, int n);
__global__ void finite_check_kernel(const float *x, int64_t n, uint32_t *flag);
__global__ void finite_check_half_kernel(const unsigned short *x, int64_t n, uint32_t *flag);
__global__ void to_half_kernel(const float *x, unsigned short *y, int64_t n);
__global__ void finalize_kernel(const double *partial, int n, DevStat *st);
__global__ void zero_kernel(uint32_t *p, int64_t n);
__global__ void shift_half_kernel(const unsigned short *x, unsigned short *y, int64_t n);
__global__ void diff_range_kernel(const double *a, const double *b, int64_t n, double *part);
__global__ void probe_read_kernel(const float4 *p, int64_t n4, int reps, float *sink);
__global__ void probe_copy_kernel(const float4 *src, float4 *dst, int64_t n4, int reps);
__global__ void restore_rows_kernel(const double *model, double *tmp, int ny, int nx, const double *b, int R);
__global__ void restore_cols_kernel(const double *tmp, const float *residual, double *out, int ny, int nx,
                                    const double *b, int R);
} // namespace cleanhip

using namespace cleanhip;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(CLEAN_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------- device -> host ----

// Small device-to-host reads (stats, flags) go through a pinned buffer of
// this thread: an asynchronous copy into pinned memory is complete once the
// stream is synchronised.  The buffer grows as needed and is kept until the
// process ends (no release from thread-exit destructors, which could run
// after the runtime has begun to shut down).
struct PinnedStage {
    void *ptr = nullptr;
    size_t bytes = 0;
};
thread_local PinnedStage t_stage;
void register_release();

// Copies n_parts (dst, src, bytes) device -> host on `stream` and waits.
// `direct`: straight into the (pageable) destinations, allocating nothing;
// the copies are complete once the stream has been synchronised.
struct D2H {
    void *dst;
    const void *src;
    size_t bytes;
};
int read_back(const D2H *parts, int n_parts, hipStream_t stream, bool direct = false)
{
    if (direct) {
        for (int i = 0; i < n_parts; ++i)
            HIPCHK(hipMemcpyAsync(parts[i].dst, parts[i].src, parts[i].bytes, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        return CLEAN_OK;
    }
    size_t total = 0;
    for (int i = 0; i < n_parts; ++i) total += align_up(parts[i].bytes, 64);
    if (t_stage.bytes < total) {
        if (t_stage.ptr) (void)hipHostFree(t_stage.ptr);
        t_stage.ptr = nullptr;
        t_stage.bytes = 0;
        const size_t sz = std::max(total, (size_t)4096);
        HIPCHK(hipHostMalloc(&t_stage.ptr, sz, hipHostMallocDefault));
        t_stage.bytes = sz;
        register_release();
    }
    size_t o = 0;
    for (int i = 0; i < n_parts; ++i) {
        HIPCHK(hipMemcpyAsync((char *)t_stage.ptr + o, parts[i].src, parts[i].bytes, hipMemcpyDeviceToHost, stream));
        o += align_up(parts[i].bytes, 64);
    }
    HIPCHK(hipStreamSynchronize(stream));
    o = 0;
    for (int i = 0; i < n_parts; ++i) {
        std::memcpy(parts[i].dst, (char *)t_stage.ptr + o, parts[i].bytes);
        o += align_up(parts[i].bytes, 64);
    }
    return CLEAN_OK;
}

// ------------------------------------------------------------ workspace --

struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
Workspace g_ws[64];
size_t g_ws_limit = 0;            // clean_set_workspace_limit (0: none)

// The library's device and pinned buffers are released at process exit, by
// a handler registered after the HIP runtime is up (so it runs before the
// runtime's own teardown): the internal workspaces and this thread's pinned
// stage.  Buffers of other threads' stages stay to the end of the process.
void release_at_exit()
{
    for (Workspace &w : g_ws)
        if (w.ptr) {
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
    if (t_stage.ptr) {
        (void)hipHostFree(t_stage.ptr);
        t_stage.ptr = nullptr;
        t_stage.bytes = 0;
    }
}
std::once_flag g_exit_once;
void register_release() { std::call_once(g_exit_once, [] { std::atexit(release_at_exit); }); }

int internal_workspace(int dev, size_t need, void **out)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    if (dev < 0 || dev >= 64) return fail(CLEAN_E_INVAL, "device %d out of range", dev);
    if (g_ws_limit && need > g_ws_limit)
        return fail(CLEAN_E_NOMEM, "workspace of %zu bytes exceeds the limit of %zu bytes", need, g_ws_limit);
    Workspace &w = g_ws[dev];
    if (w.bytes < need) {
        if (w.ptr) {
            (void)hipDeviceSynchronize();
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t sz = std::max(need, (size_t)1 << 20);
        if (g_ws_limit) sz = std::min(sz, g_ws_limit);
        if (hipMalloc(&w.ptr, sz) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CLEAN_E_NOMEM, "workspace allocation of %zu bytes failed", sz);
        }
        w.bytes = sz;
        register_release();
    }
    *out = w.ptr;
    return CLEAN_OK;
}

} // namespace

// Device scratch of the allocation-free entry point clean_hogbom_noalloc: its
// whole workspace (control block, stats, exchange slots, role table, partial
// sums).  One copy per GPU, held until the process ends.  In host code this
// name is a host-side stand-in, not a device address: only the address
// hipGetSymbolAddress returns for the current device is ever used.
static __device__ __align__(256) unsigned char scratch[CLEAN_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[64];

// The device address of `scratch` on device `dev` (the current device),
// looked up once per device.
int scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= 64) return fail(CLEAN_E_INVAL, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(CLEAN_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CLEAN_OK;
}

// Layout of one call's workspace.  The header part (control block, stats,
// exchange slots, tile keys, counts) is cleared before each launch.
struct Layout {
    size_t ctl, dstat, xslots, lslots, hslots, tile_key, rb_n, ag_n, header_end;
    size_t role, rb_idx, rb_flux, ag_pos, ag_flux, accbuf, partial;
    size_t fft_b, fft_wx, fft_wy, fft_ks, comp_img, tw_x, tw_y, rstart, psf1, total;
};

int ceil_log2(int64_t v)
{
    int lg = 0;
    while (((int64_t)1 << lg) < v) ++lg;
    return lg;
}

// FFT feedback geometry: transform sizes and which axes take two levels.
struct FftGeom {
    int lgx = 0, lgy = 0;       // 0: direct gather
    bool two_x = false, two_y = false;
};

// Slots per XCD of the two-level exchange of a plain cluster of cs
// workgroups (0: the cluster exchanges in one level).
int two_level_pad(bool tiled, int cs)
{
    return !tiled && cs >= TWO_LEVEL_MIN_CS ? ((cs + 7) / 8 + 31) / 32 * 32 : 0;
}

Layout make_layout(int T, int cs, int slot_pad, int interval, int W, int64_t npix, bool tiled, int ny = 0,
                   const FftGeom &g = FftGeom(), size_t psf1_bytes = 0)
{
    const int hpad = two_level_pad(tiled, cs);
    Layout L{};
    size_t o = 0;
    L.ctl = o;       o = align_up(o + sizeof(DevCtl), 256);
    L.dstat = o;     o = align_up(o + sizeof(DevStat), 256);
    L.xslots = o;    o = align_up(o + (size_t)T * 2 * slot_pad * 8, 256);
    L.lslots = o;    o = align_up(o + (size_t)T * 2 * slot_pad * 8, 256);
    L.hslots = o;    o = align_up(o + (hpad ? (size_t)2 * (8 * hpad + 32) * 8 : 0), 256);
    L.tile_key = o;  o = align_up(o + (size_t)T * 8, 256);
    L.rb_n = o;      o = align_up(o + (size_t)T * 4, 256);
    L.ag_n = o;      o = align_up(o + (size_t)T * 4, 256);
    L.header_end = o;
    L.role = o;      o = align_up(o + (size_t)W * 4, 256);
    const size_t list = tiled ? (size_t)T * interval * 4 : 0;
    L.rb_idx = o;    o = align_up(o + list, 256);
    L.rb_flux = o;   o = align_up(o + list, 256);
    L.ag_pos = o;    o = align_up(o + list, 256);
    L.ag_flux = o;   o = align_up(o + list, 256);
    L.accbuf = o;    o = align_up(o + (tiled ? (size_t)npix * 4 : 0), 256);
    L.partial = o;   o = align_up(o + (size_t)T * cs * 8, 256);
    const bool fft = g.lgx > 0;
    const size_t Lx = fft ? (size_t)1 << g.lgx : 0, Ly = fft ? (size_t)1 << g.lgy : 0;
    const size_t Hx = fft ? Lx / 2 + 1 : 0, rows = std::max<size_t>(ny, Ly);
    L.fft_b = o;     o = align_up(o + Hx * rows * 8, 256);
    L.fft_wx = o;    o = align_up(o + (g.two_x ? (rows + 1) / 2 * Lx * 8 : 0), 256);
    L.fft_wy = o;    o = align_up(o + (g.two_y ? Hx * Ly * 8 : 0), 256);
    L.fft_ks = o;    o = align_up(o + Hx * Ly * 8, 256);
    L.comp_img = o;  o = align_up(o + (g.two_x ? (size_t)npix * 4 : 0), 256);
    L.tw_x = o;      o = align_up(o + Lx * 8, 256);
    L.tw_y = o;      o = align_up(o + Ly * 8, 256);
    L.rstart = o;    o = align_up(o + (fft ? (size_t)npix * 4 : 0), 256);
    L.psf1 = o;      o = align_up(o + psf1_bytes, 256);
    L.total = o;
    return L;
}

// ---------------------------------------------------------- kernel table --

using KFn = void (*)(const KArgs);

template <int V, typename PT> KFn plain_fn(int K)
{
    if constexpr (V == 4) {
        switch (K) {
        case 1: return hogbom_kernel<RegTile<1, 4, PT>>;
        case 2: return hogbom_kernel<RegTile<2, 4, PT>>;
        case 4: return hogbom_kernel<RegTile<4, 4, PT>>;
        case 8: return hogbom_kernel<RegTile<8, 4, PT>>;
        case 16: return hogbom_kernel<RegTile<16, 4, PT>>;
        }
    } else {
        switch (K) {
        case 4: return hogbom_kernel<RegTile<4, 1, PT>>;
        case 16: return hogbom_kernel<RegTile<16, 1, PT>>;
        case 32: return hogbom_kernel<RegTile<32, 1, PT>>;
        }
    }
    return nullptr;
}

template <int V, typename PT, bool FFT> KFn tiled_fn(int K)
{
    if constexpr (V == 4) {
        switch (K) {
        case 1: return tiled_kernel<RegTile<1, 4, PT>, FFT>;
        case 2: return tiled_kernel<RegTile<2, 4, PT>, FFT>;
        case 4: return tiled_kernel<RegTile<4, 4, PT>, FFT>;
        case 8: return tiled_kernel<RegTile<8, 4, PT>, FFT>;
        case 16: return tiled_kernel<RegTile<16, 4, PT>, FFT>;
        }
    } else {
        switch (K) {
        case 4: return tiled_kernel<RegTile<4, 1, PT>, FFT>;
        case 16: return tiled_kernel<RegTile<16, 1, PT>, FFT>;
        case 32: return tiled_kernel<RegTile<32, 1, PT>, FFT>;
        }
    }
    return nullptr;
}

template <int V, typename PT> KFn tiled_fn(int K, bool fft)
{
    return fft ? tiled_fn<V, PT, true>(K) : tiled_fn<V, PT, false>(K);
}

using BFn = void (*)(const BatchArgs);

template <int V, typename PT, bool TILED> BFn batched_fn(int K)
{
    if constexpr (V == 4) {
        switch (K) {
        case 1: return batched_kernel<RegTile<1, 4, PT>, TILED>;
        case 2: return batched_kernel<RegTile<2, 4, PT>, TILED>;
        case 4: return batched_kernel<RegTile<4, 4, PT>, TILED>;
        case 8: return batched_kernel<RegTile<8, 4, PT>, TILED>;
        case 16: return batched_kernel<RegTile<16, 4, PT>, TILED>;
        }
    } else {
        switch (K) {
        case 4: return batched_kernel<RegTile<4, 1, PT>, TILED>;
        case 16: return batched_kernel<RegTile<16, 1, PT>, TILED>;
        case 32: return batched_kernel<RegTile<32, 1, PT>, TILED>;
        }
    }
    return nullptr;
}

// The batched kernel for this PSF dtype, group width and pixels per thread;
// `tiled`: the variant that also runs tiled problems (more registers, so it
// is used only for batches that hold one).
BFn pick_batched(bool half, int V, int K, bool tiled)
{
    if (tiled) {
        if (V == 4) return half ? batched_fn<4, __half, true>(K) : batched_fn<4, float, true>(K);
        return half ? batched_fn<1, __half, true>(K) : batched_fn<1, float, true>(K);
    }
    if (V == 4) return half ? batched_fn<4, __half, false>(K) : batched_fn<4, float, false>(K);
    return half ? batched_fn<1, __half, false>(K) : batched_fn<1, float, false>(K);
}

KFn pick_wide(bool half, bool fft)
{
    if (fft) return half ? tiled_kernel<WideTile<__half>, true> : tiled_kernel<WideTile<float>, true>;
    return half ? tiled_kernel<WideTile<__half>, false> : tiled_kernel<WideTile<float>, false>;
}

template <bool FFT> KFn tiled_stream_fn(bool half, int V)
{
    if (V == 4) return half ? tiled_kernel<StreamTile<STREAM_K, 4, __half>, FFT> : tiled_kernel<StreamTile<STREAM_K, 4, float>, FFT>;
    return half ? tiled_kernel<StreamTile<STREAM_K, 1, __half>, FFT> : tiled_kernel<StreamTile<STREAM_K, 1, float>, FFT>;
}

KFn pick_stream(bool tiled, bool half, int V, bool fft)
{
    if (tiled) return fft ? tiled_stream_fn<true>(half, V) : tiled_stream_fn<false>(half, V);
    if (V == 4) return half ? hogbom_kernel<StreamTile<STREAM_K, 4, __half>> : hogbom_kernel<StreamTile<STREAM_K, 4, float>>;
    return half ? hogbom_kernel<StreamTile<STREAM_K, 1, __half>> : hogbom_kernel<StreamTile<STREAM_K, 1, float>>;
}

KFn pick(bool tiled, bool half, int V, int K, bool fft)
{
    if (tiled) {
        if (V == 4) return half ? tiled_fn<4, __half>(K, fft) : tiled_fn<4, float>(K, fft);
        return half ? tiled_fn<1, __half>(K, fft) : tiled_fn<1, float>(K, fft);
    }
    if (V == 4) return half ? plain_fn<4, __half>(K) : plain_fn<4, float>(K);
    return half ? plain_fn<1, __half>(K) : plain_fn<1, float>(K);
}

bool valid_ppt(int V, int ppt)
{
    if (V == 4) return ppt == 4 || ppt == 8 || ppt == 16 || ppt == 32 || ppt == 64;
    return ppt == 4 || ppt == 16 || ppt == 32;
}

// Launch shape for a tile of npix pixels: workgroups per cluster (cs) and
// pixels per thread (ppt = K*V).  Small clusters keep the per-iteration
// exchange short; the pixels per thread bound each workgroup's PSF traffic.
// xcd_clusters > 0 (tiled launches: clusters per XCD) asks for the XCD-local
// exchange: the smallest ppt whose clusters, xcd_clusters of them, fit one
// XCD's xcd_cus CUs at one workgroup each.  Their exchanges stay in that
// XCD's L2, cheap enough that more, smaller workgroups win (1024^2 in 2 x 2
// tiles: 16 px/thread x 32 workgroups 13.2 ms, 32 x 16 15.5 ms; 512^2:
// 4 x 32 10.6 ms, 32 x 4 13.9 ms).
int choose_shape(int64_t npix, int V, int user_cs, int user_ppt, int max_ppt, int xcd_clusters, int xcd_cus,
                 int &cs, int &ppt)
{
    if (user_ppt) {
        if (!valid_ppt(V, user_ppt))
            return fail(CLEAN_E_INVAL, "px_per_thread %d not available (tile width %s a multiple of 4)", user_ppt,
                        V == 4 ? "is" : "is not");
        ppt = user_ppt;
        cs = user_cs ? user_cs : (int)((npix + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
    } else if (user_cs) {
        cs = user_cs;
        const int opts4[] = {4, 8, 16, 32, 64}, opts1[] = {4, 16, 32};
        const int *opts = V == 4 ? opts4 : opts1;
        int nopt = V == 4 ? 5 : 3;
        while (nopt > 1 && opts[nopt - 1] > max_ppt) --nopt;
        ppt = opts[nopt - 1];
        for (int i = 0; i < nopt; ++i)
            if ((int64_t)cs * WG * opts[i] >= npix) { ppt = opts[i]; break; }
    } else if (xcd_clusters == 0 && V == 4 && npix > (int64_t)WG * 4) {
        // plain CLEAN: one cluster over the whole device.  Up to 64K pixels, 16
        // px/thread in at most 8 workgroups (a one-level exchange); above, 8
        // px/thread and as many workgroups as that takes, up to 512 (two
        // workgroups per CU), with more pixels per thread beyond (256^2: 8 x 16
        // 2.19 ms against 4 x 32 2.39 ms and 16 x 8 3.12 ms; 1024^2: 256 x 8
        // 71.2 ms against 128 x 16 75.1 ms and 64 x 32 84.6 ms, 20000
        // iterations)
        if (npix <= (int64_t)8 * WG * 16) {
            ppt = 16;
        } else {
            ppt = 8;
            while ((npix + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt) > 512 && ppt * 2 <= max_ppt) ppt *= 2;
        }
        cs = (int)((npix + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
    } else {
        const int opts4[] = {4, 8, 16, 32, 64}, opts1[] = {4, 16, 32};
        const int *opts = V == 4 ? opts4 : opts1;
        int nopt = V == 4 ? 5 : 3;
        while (nopt > 1 && opts[nopt - 1] > max_ppt) --nopt;
        // smallest ppt that fits one workgroup, else 32 px/thread with as many
        // workgroups as needed, growing ppt (up to max_ppt) when clusters get large
        ppt = 0;
        for (int i = 0; i < nopt; ++i)
            if ((int64_t)WG * opts[i] >= npix) { ppt = opts[i]; cs = 1; break; }
        if (!ppt && xcd_clusters > 0) {
            for (int i = 0; i < nopt; ++i) {
                const int64_t c = (npix + (int64_t)WG * opts[i] - 1) / ((int64_t)WG * opts[i]);
                if (c * xcd_clusters <= xcd_cus) { ppt = opts[i]; cs = (int)c; break; }
            }
        }
        if (!ppt) {
            // 32 px/thread measured fastest up to 64 workgroups per cluster
            ppt = std::min(V == 4 ? 32 : 16, max_ppt);
            cs = (int)((npix + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
            while (cs > 64 && ppt < opts[nopt - 1]) {
                for (int i = 0; i < nopt; ++i)
                    if (opts[i] > ppt) { ppt = opts[i]; break; }
                cs = (int)((npix + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
            }
        }
    }
    if ((int64_t)cs * WG * ppt < npix)
        return fail(CLEAN_E_INVAL, "launch shape %d workgroups x %d px/thread cannot hold %lld pixels", cs, ppt,
                    (long long)npix);
    if (cs < 1 || cs > 4096) return fail(CLEAN_E_UNSUPPORTED, "cluster of %d workgroups not supported", cs);
    return CLEAN_OK;
}

int device_timeout_ticks(int dev, uint64_t &ticks)
{
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) khz = 100000;
    ticks = (uint64_t)khz * 1000ull * 20ull;     // 20 seconds per wait
    return CLEAN_OK;
}

// Transform sizes for FFT feedback: powers of two >= 2n - 1 per axis; an axis
// longer than 8192 points (or any axis of length >= 4, when asked) takes two
// levels.
int fft_geometry(int ny, int nx, int flags, FftGeom &g)
{
    g.lgx = std::max(1, ceil_log2(2 * (int64_t)nx - 1));
    g.lgy = std::max(1, ceil_log2(2 * (int64_t)ny - 1));
    if (g.lgx > FFT_MAX_LG2 || g.lgy > FFT_MAX_LG2)
        return fail(CLEAN_E_UNSUPPORTED, "FFT feedback supports images up to 32768 x 32768 (transforms of 65536)");
    const bool force = flags & CLEAN_FLAG_FFT_TWO_LEVEL;
    g.two_x = g.lgx > FFT_MAX_LG || (force && g.lgx >= 2);
    g.two_y = g.lgy > FFT_MAX_LG || (force && g.lgy >= 2);
    return CLEAN_OK;
}

int check_common(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx, const clean_params *p,
                 float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap)
{
    if (!p) return fail(CLEAN_E_INVAL, "params is NULL");
    if (!dirty || !psf || !residual) return fail(CLEAN_E_INVAL, "dirty, psf and residual must be non-NULL");
    if (comp_cap > 0 && (!comp_idx || !comp_flux)) return fail(CLEAN_E_INVAL, "component arrays are NULL");
    if (ny <= 0 || nx <= 0) return fail(CLEAN_E_INVAL, "image size %d x %d", ny, nx);
    if ((int64_t)ny * nx > (1ll << 28)) return fail(CLEAN_E_UNSUPPORTED, "image of %lld pixels exceeds 2^28", (long long)ny * nx);
    if (psf_ny < 2 * (int64_t)ny || psf_nx < 2 * (int64_t)nx)
        return fail(CLEAN_E_INVAL, "PSF %d x %d must be at least twice the image %d x %d", psf_ny, psf_nx, ny, nx);
    const uint64_t es = p->psf_dtype == CLEAN_PSF_F16 ? 2 : 4;
    if ((uint64_t)psf_ny * psf_nx * es > (1ull << 34)) return fail(CLEAN_E_UNSUPPORTED, "PSF larger than 16 GiB");
    if ((uint64_t)((int64_t)(ny - 1) * psf_nx + nx) * es > 0xFFFFFFFFull)
        return fail(CLEAN_E_UNSUPPORTED, "image x PSF row length too large for 32-bit offsets");
    if (!(p->gain > 0.0 && p->gain <= 1.0)) return fail(CLEAN_E_INVAL, "gain %g not in (0, 1]", p->gain);
    if (!(p->threshold >= 0.0)) return fail(CLEAN_E_INVAL, "threshold %g < 0", p->threshold);
    if (p->max_iter < 0) return fail(CLEAN_E_INVAL, "max_iter %lld < 0", (long long)p->max_iter);
    if (comp_cap < 0) return fail(CLEAN_E_INVAL, "comp_cap < 0");
    if (p->psf_dtype != CLEAN_PSF_F32 && p->psf_dtype != CLEAN_PSF_F16)
        return fail(CLEAN_E_INVAL, "psf_dtype %d", p->psf_dtype);
    if (p->wg_per_tile < 0 || p->px_per_thread < 0) return fail(CLEAN_E_INVAL, "negative launch shape");
    return CLEAN_OK;
}

// Shared driver of the plain and tiled forms.
// noalloc: the workspace is the device scratch array (the allocation-free
// entry point): nothing is allocated, the header is cleared by a fill kernel,
// results come back by direct copies, and the call is not timed.
int run(bool tiled, const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx, int tiles_y,
        int tiles_x, int interval, const clean_params *p, float *residual, int32_t *comp_idx, float *comp_flux,
        int64_t comp_cap, double *model, void *workspace, size_t workspace_bytes, clean_stats *stats,
        void *stream_v, bool noalloc = false)
{
    int st = check_common(dirty, ny, nx, psf, psf_ny, psf_nx, p, residual, comp_idx, comp_flux, comp_cap);
    if (st) return st;
    if (tiled) {
        if (tiles_y < 1 || tiles_x < 1 || tiles_y > ny || tiles_x > nx)
            return fail(CLEAN_E_INVAL, "tile grid %d x %d for a %d x %d image", tiles_y, tiles_x, ny, nx);
        if ((int64_t)tiles_y * tiles_x > MAX_TILES)
            return fail(CLEAN_E_UNSUPPORTED, "%d tiles exceed %d", tiles_y * tiles_x, MAX_TILES);
        if (interval < 1 || interval > MAX_INTERVAL)
            return fail(CLEAN_E_INVAL, "feedback interval %d not in [1, %d]", interval, MAX_INTERVAL);
        if (!(p->feedback_level >= 0.0 && p->feedback_level <= 1.0))
            return fail(CLEAN_E_INVAL, "feedback_level %g not in [0, 1]", p->feedback_level);
        if (!(p->flags & CLEAN_FLAG_FFT_FEEDBACK)) {
            // worst case of one round's direct gather: every tile appends
            // `interval` distinct components, each read over every pixel
            // outside its tile
            const int64_t smallest = (int64_t)(ny / tiles_y) * (nx / tiles_x);
            const double worst = (double)tiles_y * tiles_x * interval * (double)((int64_t)ny * nx - smallest) *
                                 (p->psf_dtype == CLEAN_PSF_F16 ? 2.0 : 4.0);
            if (worst > GATHER_MAX_BYTES)
                return fail(CLEAN_E_UNSUPPORTED, "a round of direct-gather feedback could read %.3g bytes of PSF, "
                            "more than a round may take within the device's wait limit; use "
                            "CLEAN_FLAG_FFT_FEEDBACK", worst);
        }
    } else {
        tiles_y = tiles_x = 1;
        interval = 1;
    }
    const bool fft = tiled && (p->flags & CLEAN_FLAG_FFT_FEEDBACK);
    FftGeom fg;
    if (fft) {
        st = fft_geometry(ny, nx, p->flags, fg);
        if (st) return st;
    }
    hipStream_t stream = (hipStream_t)stream_v;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

    const int T = tiles_y * tiles_x;
    // tile geometry: widths all multiples of 4 allow 4-wide pixel groups
    int64_t max_tile = 0;
    bool w4 = true;
    for (int i = 0; i < tiles_y; ++i)
        for (int j = 0; j < tiles_x; ++j) {
            const int h = (int)((int64_t)(i + 1) * ny / tiles_y - (int64_t)i * ny / tiles_y);
            const int w = (int)((int64_t)(j + 1) * nx / tiles_x - (int64_t)j * nx / tiles_x);
            max_tile = std::max<int64_t>(max_tile, (int64_t)h * w);
            if (w % 4) w4 = false;
        }
    const int V = w4 ? 4 : 1;
    const bool half = p->psf_dtype == CLEAN_PSF_F16;
    size_t dyn_lds = tiled ? std::max((size_t)16 * ((interval + 3) & ~3), (size_t)8 * GATHER_CHUNK) : 0;
    if (fft) {
        if (!fg.two_x) dyn_lds = std::max(dyn_lds, (size_t)8 * fft_pad_slots(1 << fg.lgx));
        if (!fg.two_y) dyn_lds = std::max(dyn_lds, (size_t)8 * fft_pad_slots(1 << fg.lgy));
        if (fg.two_x || fg.two_y) dyn_lds = std::max(dyn_lds, (size_t)8 * FFT_LDS_CPLX);
    }

    // placement: cluster c lives on XCD c % 8 (workgroup b runs on XCD b % 8);
    // tiled launches add helper workgroups for the feedback gather.  There is
    // one cluster per tile, except for the time-multiplexed wide tile, whose
    // nclusters clusters each run several tiles in turn.
    int nclusters = T;
    auto place = [&](int cs, int max_wg, int &W, std::vector<int32_t> &role) -> bool {
        if (!tiled) {
            W = cs;
            if (W > max_wg) return false;
            role.resize(W);
            for (int b = 0; b < W; ++b) role[b] = b;
            return true;
        }
        std::vector<int> need(8, 0);
        for (int c = 0; c < nclusters; ++c) need[c % 8] += cs;
        W = 8 * *std::max_element(need.begin(), need.end());
        const int helpers_target = std::min(max_wg, 2 * ncu) / 8 * 8;
        if (W < helpers_target) W = helpers_target;
        if (W > max_wg) {
            W = nclusters * cs;              // pack without XCD affinity
            if (W > max_wg) return false;
            role.assign(W, -1);
            for (int c = 0; c < nclusters; ++c)
                for (int g = 0; g < cs; ++g) role[c * cs + g] = (c << 16) | g;
            return true;
        }
        role.assign(W, -1);
        std::vector<int> fill(8, 0);
        for (int c = 0; c < nclusters; ++c) {
            const int x = c % 8;
            for (int g = 0; g < cs; ++g) role[x + 8 * fill[x]++] = (c << 16) | g;
        }
        return true;
    };

    // register-resident residual when the launch fits, else streamed through HBM
    int cs = 0, ppt = 0, W = 0;
    bool streamed = false;
    KFn fn = nullptr;
    std::vector<int32_t> role;
    const bool force_stream = (p->flags & CLEAN_FLAG_STREAM_RESIDUAL) != 0;
    if (force_stream && p->px_per_thread)
        return fail(CLEAN_E_INVAL, "px_per_thread applies to the register-resident form only");
    const bool want_wide = tiled && p->px_per_thread == 128;   // the wide tile on request
    if (want_wide && p->wg_per_tile)
        return fail(CLEAN_E_INVAL, "px_per_thread = 128 (the wide tile) picks its own workgroups per tile");
    st = force_stream || want_wide ? CLEAN_E_UNSUPPORTED
                      : choose_shape(max_tile, V, p->wg_per_tile, p->px_per_thread, tiled ? 32 : 64,
                                     tiled ? (T + 7) / 8 : 0, ncu / 8, cs, ppt);
    // the allocation-free entry point refuses a cluster whose workspace does
    // not fit its scratch array before anything else (plain: W = cs)
    auto noalloc_fits = [&](int c) -> int {
        if (!noalloc) return CLEAN_OK;
        const size_t need = make_layout(1, c, (c + 31) / 32 * 32, 1, c, (int64_t)ny * nx, false).total;
        if (need > CLEAN_NOALLOC_SCRATCH_BYTES)
            return fail(CLEAN_E_UNSUPPORTED, "a cluster of %d workgroups needs %zu bytes of workspace; the "
                        "allocation-free entry point holds %d", c, need, (int)CLEAN_NOALLOC_SCRATCH_BYTES);
        return CLEAN_OK;
    };
    if (st == CLEAN_OK && (st = noalloc_fits(cs)) != CLEAN_OK) return st;
    if (st == CLEAN_OK) {
        fn = pick(tiled, half, V, ppt / V, fft);
        if (!fn) return fail(CLEAN_E_UNSUPPORTED, "no kernel for %d pixels per thread", ppt);
        if (dyn_lds > 48 * 1024)
            HIPCHK(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
        int occ = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)fn, WG, dyn_lds));
        occ = std::min(occ, MAX_WG_PER_CU);
        if (!place(cs, occ * ncu, W, role)) {
            if (p->px_per_thread)
                return fail(CLEAN_E_UNSUPPORTED, "%d x %d workgroups cannot be co-resident (max %d)", T, cs, occ * ncu);
            streamed = true;
        }
    } else if (p->px_per_thread == 0 || want_wide) {
        streamed = true;
    } else {
        return st;
    }
    // tiles too large for the register tiles: 128 px/thread held in registers
    // during the local loops (WideTile) when the image fits the co-resident
    // register file that way, else the residual streamed through HBM
    if (streamed && !force_stream && tiled && V == 4 && !p->wg_per_tile && (!p->px_per_thread || want_wide) &&
        nx % tiles_x == 0) {
        const int tw = nx / tiles_x;
        const int64_t per_wg = (int64_t)WG * 128;
        const int cw = (int)((max_tile + per_wg - 1) / per_wg);
        if (((int64_t)cw * WG * 4) % tw == 0) {
            KFn fw = pick_wide(half, fft);
            size_t wide_lds = dyn_lds;
            if (fft) {
                // its padded one-level arenas
                if (!fg.two_x) wide_lds = std::max(wide_lds, (size_t)8 * fft_pad_slots(1 << fg.lgx));
                if (!fg.two_y) wide_lds = std::max(wide_lds, (size_t)8 * fft_pad_slots(1 << fg.lgy));
            }
            if (wide_lds > 48 * 1024)
                HIPCHK(hipFuncSetAttribute((const void *)fw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)wide_lds));
            int occ = 0;
            HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)fw, WG, wide_lds));
            occ = std::min(occ, MAX_WG_PER_CU);
            if (occ > 0 && place(cw, occ * ncu, W, role)) {
                streamed = false;
                fn = fw;
                cs = cw;
                ppt = 128;
                dyn_lds = wide_lds;
            } else if (occ > 0 && (want_wide || max_tile >= (int64_t)WG * 128)) {
                // time-multiplexed: as many clusters as one XCD's share of the
                // co-resident workgroups holds, eight XCDs' worth, each cluster
                // running its tiles in turn in every round (tiles of at least
                // one wide workgroup's pixels, or on request)
                const int nc = std::min(T, 8 * ((occ * ncu / 8) / cw));
                if (nc >= 1) {
                    nclusters = nc;
                    if (place(cw, occ * ncu, W, role)) {
                        streamed = false;
                        fn = fw;
                        cs = cw;
                        ppt = 128;
                        dyn_lds = wide_lds;
                    } else {
                        nclusters = T;
                    }
                }
            }
        }
    }
    if (want_wide && streamed)
        return fail(CLEAN_E_UNSUPPORTED, "the wide tile needs tile widths that are equal, multiples of 4 and "
                                         "divide %d x 2048 pixels, and a co-resident launch",
                    (int)((max_tile + (int64_t)WG * 128 - 1) / ((int64_t)WG * 128)));
    if (streamed) {
        g_last_error.clear();
        fn = pick_stream(tiled, half, V, fft);
        if (dyn_lds > 48 * 1024)
            HIPCHK(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
        int occ = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)fn, WG, dyn_lds));
        occ = std::min(occ, MAX_WG_PER_CU);
        const int max_wg = occ * ncu;
        const int64_t per_wg = (int64_t)WG * STREAM_K * V;
        const int64_t need = (max_tile + per_wg - 1) / per_wg;
        if (p->wg_per_tile) cs = p->wg_per_tile;
        else cs = (int)std::max<int64_t>(1, std::min<int64_t>(need, tiled ? std::max(1, max_wg / T) : max_wg));
        ppt = 0;
        if ((st = noalloc_fits(cs)) != CLEAN_OK) return st;
        if (cs > 4096 || !place(cs, max_wg, W, role))
            return fail(CLEAN_E_UNSUPPORTED, "%d x %d streaming workgroups cannot be co-resident (max %d)", T, cs, max_wg);
    }

    const int slot_pad = (cs + 31) / 32 * 32;
    const int64_t npix = (int64_t)ny * nx;
    // the wide tile with an FP16 PSF: room for the PSF moved down one element
    // (left out when a caller's workspace has no room for it)
    const size_t psf1_bytes = tiled && half && ppt == 128 ? (size_t)psf_ny * psf_nx * 2 : 0;
    Layout L = make_layout(T, cs, slot_pad, interval, W, npix, tiled, ny, fg, psf1_bytes);
    if (psf1_bytes && workspace && !noalloc && workspace_bytes < L.total)
        L = make_layout(T, cs, slot_pad, interval, W, npix, tiled, ny, fg);
    char *ws = (char *)workspace;
    if (noalloc) {
        if (L.total > CLEAN_NOALLOC_SCRATCH_BYTES)     // not reached: noalloc_fits ran first
            return fail(CLEAN_E_UNSUPPORTED, "this launch (%d workgroups) needs %zu bytes of workspace; the "
                        "allocation-free entry point holds %d", W, L.total, (int)CLEAN_NOALLOC_SCRATCH_BYTES);
        void *sp = nullptr;
        st = scratch_address(dev, &sp);
        if (st) return st;
        ws = (char *)sp;
    } else if (ws) {
        if (workspace_bytes < L.total)
            return fail(CLEAN_E_NOMEM, "workspace of %zu bytes < %zu needed", workspace_bytes, L.total);
    } else {
        void *wp = nullptr;
        st = internal_workspace(dev, L.total, &wp);
        if (st) return st;
        ws = (char *)wp;
    }

    KArgs a{};
    a.dirty = dirty;
    a.residual = residual;
    a.model = model;
    a.psf = psf;
    a.psf_bytes = (uint64_t)psf_ny * psf_nx * (half ? 2 : 4);
    a.ny = ny; a.nx = nx; a.psf_ny = psf_ny; a.psf_nx = psf_nx;
    a.cy = psf_ny / 2; a.cx = psf_nx / 2;
    a.ty = tiles_y; a.tx = tiles_x; a.T = T;
    a.cs = cs;
    a.ncl = nclusters;
    a.slot_pad = slot_pad;
    a.interval = interval;
    a.level_frac = tiled ? p->feedback_level : 0.0;
    a.gather_parts = std::max(1, W / T);
    a.gain = (float)p->gain;
    a.threshold = p->threshold;
    a.max_iter = p->max_iter;
    a.cap = comp_cap;
    st = device_timeout_ticks(dev, a.timeout_ticks);
    if (st) return st;
    a.comp_idx = comp_idx;
    a.comp_flux = comp_flux;
    a.cancel = (const int32_t *)p->cancel;
    a.has_cancel = p->cancel != nullptr;
    a.ctl = (DevCtl *)(ws + L.ctl);
    a.bar = &a.ctl->barrier;
    a.cword = &a.ctl->cancel;
    a.dstat = (DevStat *)(ws + L.dstat);
    a.role = (const int32_t *)(ws + L.role);
    a.xslots = (uint64_t *)(ws + L.xslots);
    a.lslots = (uint64_t *)(ws + L.lslots);
    a.hpad = two_level_pad(tiled, cs);
    a.hslots = a.hpad ? (uint64_t *)(ws + L.hslots) : nullptr;
    a.tile_key = (uint64_t *)(ws + L.tile_key);
    a.rb_idx = (int32_t *)(ws + L.rb_idx);
    a.rb_flux = (float *)(ws + L.rb_flux);
    a.rb_n = (int32_t *)(ws + L.rb_n);
    a.ag_pos = (int32_t *)(ws + L.ag_pos);
    a.ag_flux = (float *)(ws + L.ag_flux);
    a.ag_n = (int32_t *)(ws + L.ag_n);
    a.accbuf = (float *)(ws + L.accbuf);
    a.partial = (double *)(ws + L.partial);
    a.fft_lgx = fg.lgx;
    a.fft_lgy = fg.lgy;
    a.fft_two_x = fg.two_x;
    a.fft_two_y = fg.two_y;
    a.fft_b = (float2 *)(ws + L.fft_b);
    a.fft_wx = (float2 *)(ws + L.fft_wx);
    a.fft_wy = (float2 *)(ws + L.fft_wy);
    a.fft_ks = (float2 *)(ws + L.fft_ks);
    a.comp_img = fg.two_x ? (float *)(ws + L.comp_img) : nullptr;
    a.tw_x = (const float2 *)(ws + L.tw_x);
    a.tw_y = (const float2 *)(ws + L.tw_y);
    a.rstart = fft ? (float *)(ws + L.rstart) : nullptr;
    a.psf1 = L.psf1 != L.total && psf1_bytes && L.total - L.psf1 >= psf1_bytes ? (const void *)(ws + L.psf1) : nullptr;

    if (noalloc) {
        // the header is a whole number of 256-byte blocks
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, stream, (uint32_t *)ws, (int64_t)(L.header_end / 4));
        HIPCHK(hipGetLastError());
    } else {
        HIPCHK(hipMemsetAsync(ws, 0, L.header_end, stream));
    }
    HIPCHK(hipMemcpyAsync(ws + L.role, role.data(), role.size() * 4, hipMemcpyHostToDevice, stream));
    if (p->flags & CLEAN_FLAG_CHECK_FINITE) {
        uint32_t *flag = &a.ctl->finite_bad;
        hipLaunchKernelGGL(finite_check_kernel, dim3(1024), dim3(256), 0, stream, dirty, npix, flag);
        if (half)
            hipLaunchKernelGGL(finite_check_half_kernel, dim3(1024), dim3(256), 0, stream,
                               (const unsigned short *)psf, (int64_t)psf_ny * psf_nx, flag);
        else
            hipLaunchKernelGGL(finite_check_kernel, dim3(1024), dim3(256), 0, stream, (const float *)psf,
                               (int64_t)psf_ny * psf_nx, flag);
        HIPCHK(hipGetLastError());
        uint32_t bad = 0;
        const D2H rb[1] = {{&bad, flag, 4}};
        st = read_back(rb, 1, stream, noalloc);
        if (st) return st;
        if (bad) return fail(CLEAN_E_NONFINITE, "non-finite value in the dirty image or PSF");
    }

    if (a.psf1) {
        hipLaunchKernelGGL(shift_half_kernel, dim3(2048), dim3(256), 0, stream, (const unsigned short *)psf,
                           (unsigned short *)a.psf1, (int64_t)psf_ny * psf_nx);
        HIPCHK(hipGetLastError());
    }

    std::vector<float2> twx, twy;
    if (fft) {
        // twiddles W_L^m = exp(-2 pi i m / L), m < L, in double, rounded once;
        // the PSF kernel's spectrum is computed at the start of the launch
        for (int pass = 0; pass < 2; ++pass) {
            const int lg = pass ? fg.lgy : fg.lgx;
            std::vector<float2> &tw = pass ? twy : twx;
            const int Lt = 1 << lg;
            tw.resize(Lt);
            for (int m = 0; m < Lt; ++m) {
                const double ang = -2.0 * M_PI * (double)m / (double)Lt;
                tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
            }
        }
        HIPCHK(hipMemcpyAsync(ws + L.rstart, dirty, (size_t)npix * 4, hipMemcpyDeviceToDevice, stream));
        if (fg.two_x) HIPCHK(hipMemsetAsync(ws + L.comp_img, 0, (size_t)npix * 4, stream));
        HIPCHK(hipMemcpyAsync(ws + L.tw_x, twx.data(), twx.size() * 8, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(ws + L.tw_y, twy.data(), twy.size() * 8, hipMemcpyHostToDevice, stream));
    }

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!noalloc) {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, stream));
    }
    void *args[] = {(void *)&a};
    hipError_t le = hipLaunchCooperativeKernel((const void *)fn, dim3(W), dim3(WG), args, (unsigned)dyn_lds, stream);
    if (le != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(CLEAN_E_HIP, "cooperative launch of %d x %d failed: %s", W, WG, hipGetErrorString(le));
    }
    if (!noalloc) HIPCHK(hipEventRecord(e1, stream));
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, stream, a.partial, T * cs, a.dstat);
    HIPCHK(hipGetLastError());
    DevStat ds{};
    DevCtl ctl{};
    const D2H rb[2] = {{&ds, a.dstat, sizeof ds}, {&ctl, a.ctl, sizeof ctl}};
    st = read_back(rb, 2, stream, noalloc);
    if (st) return st;
    float ms = 0.f;
    if (!noalloc) {
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (ctl.abort & ABORT_TIMEOUT) return fail(CLEAN_E_TIMEOUT, "a device-side wait timed out");
    if (ctl.abort) return fail(CLEAN_E_HIP, "device abort code %u", ctl.abort);
    if (stats) {
        stats->n_iter = ds.n_iter;
        stats->stop_reason = ds.stop;
        stats->n_rounds = ds.n_rounds;
        stats->final_peak = ds.final_peak;
        stats->residual_rms = std::sqrt(ds.sumsq / (double)npix);
        stats->model_flux = ds.model_flux;
        stats->device_ms = ms;
        stats->wg_per_tile = cs;
        stats->px_per_thread = ppt;
        stats->workgroups = W;
        stats->streamed = streamed;
        stats->xcd_local_clusters = ds.xcd_local;
        stats->exchange_levels = ds.levels > 0 ? ds.levels : 1;
        const double us_per_tick = 1e6 / (double)(a.timeout_ticks / 20ull);
        for (int i = 0; i < 3; ++i) stats->phase_us[i] = (float)(ds.phase_ticks[i] * us_per_tick);
    }
    return CLEAN_OK;
}

} // namespace

extern "C" {

int clean_hogbom(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx, const clean_params *p,
                 float *residual, int32_t *comp_idx, float *comp_flux, int64_t comp_cap, double *model,
                 void *workspace, size_t workspace_bytes, clean_stats *stats, void *stream)
{
    g_last_error.clear();
    return run(false, dirty, ny, nx, psf, psf_ny, psf_nx, 1, 1, 1, p, residual, comp_idx, comp_flux, comp_cap, model,
               workspace, workspace_bytes, stats, stream);
}

int clean_hogbom_noalloc(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                         const clean_params *p, float *residual, int32_t *comp_idx, float *comp_flux,
                         int64_t comp_cap, double *model, clean_stats *stats, void *stream)
{
    g_last_error.clear();
    return run(false, dirty, ny, nx, psf, psf_ny, psf_nx, 1, 1, 1, p, residual, comp_idx, comp_flux, comp_cap, model,
               nullptr, 0, stats, stream, true);
}

int clean_tiled_feedback(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx, int tiles_y,
                         int tiles_x, int feedback_interval, const clean_params *p, float *residual,
                         int32_t *comp_idx, float *comp_flux, int64_t comp_cap, double *model, void *workspace,
                         size_t workspace_bytes, clean_stats *stats, void *stream)
{
    g_last_error.clear();
    return run(true, dirty, ny, nx, psf, psf_ny, psf_nx, tiles_y, tiles_x, feedback_interval, p, residual, comp_idx,
               comp_flux, comp_cap, model, workspace, workspace_bytes, stats, stream);
}

namespace {
// Launch shapes chosen by clean_autotune_batched, per process, keyed by the
// device and a signature of the batch: the PSF dtype, the flags and every
// problem's image, PSF and tile-grid sizes and interval, in order (FNV-1a).
std::mutex g_btune_mu;
std::map<std::pair<int, uint64_t>, int> g_btune_cache;

uint64_t batch_signature(const clean_problem *probs, int n, const clean_params *p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)(v >> (8 * b)) & 0xFFu;
            h *= 1099511628211ull;
        }
    };
    mix(n);
    mix(p->psf_dtype);
    mix(p->flags);
    for (int i = 0; i < n; ++i) {
        const clean_problem &q = probs[i];
        mix(q.ny);
        mix(q.nx);
        mix(q.psf_ny);
        mix(q.psf_nx);
        mix(q.tiles_y);
        mix(q.tiles_x);
        mix(q.tiles_y * q.tiles_x > 1 ? q.interval : 0);
    }
    return h;
}

// 4 when every tile of every problem is a multiple of 4 pixels wide (the
// batched kernels' 4-wide groups), else 1: the rule clean_batched applies.
int batch_group_width(const clean_problem *probs, int n)
{
    for (int i = 0; i < n; ++i) {
        const int tx = probs[i].tiles_x > 0 ? probs[i].tiles_x : 1;
        for (int b = 0; b < tx; ++b)
            if ((int)((int64_t)(b + 1) * probs[i].nx / tx - (int64_t)b * probs[i].nx / tx) % 4) return 1;
    }
    return 4;
}

bool btune_lookup(int dev, uint64_t sig, int &ppt)
{
    std::lock_guard<std::mutex> lk(g_btune_mu);
    auto it = g_btune_cache.find({dev, sig});
    if (it == g_btune_cache.end()) return false;
    ppt = it->second;
    return true;
}
}   // namespace

int clean_batched(const clean_problem *probs, int n, const clean_params *shared, clean_stats *stats, void *stream_v)
{
    g_last_error.clear();
    if (!probs || !shared) return fail(CLEAN_E_INVAL, "probs and shared params must be non-NULL");
    if (n < 0 || n > 65536) return fail(CLEAN_E_INVAL, "batch of %d problems not in [0, 65536]", n);
    if (n == 0) return CLEAN_OK;
    if (shared->flags & CLEAN_FLAG_FFT_FEEDBACK)
        return fail(CLEAN_E_UNSUPPORTED, "tiled problems of a batch use the direct gather (no CLEAN_FLAG_FFT_FEEDBACK)");
    if (!(shared->feedback_level >= 0.0 && shared->feedback_level <= 1.0))
        return fail(CLEAN_E_INVAL, "feedback_level %g not in [0, 1]", shared->feedback_level);
    const bool half = shared->psf_dtype == CLEAN_PSF_F16;
    // per problem: tile grid (1 x 1: plain), the largest tile, 4-wide groups
    std::vector<int> pty(n, 1), ptx(n, 1), pint(n, 1);
    std::vector<int64_t> ptile(n, 0);
    bool w4 = true, any_tiled = false;
    int max_interval = 1;
    for (int i = 0; i < n; ++i) {
        const clean_problem &q = probs[i];
        clean_params pi = *shared;
        pi.threshold = q.threshold;
        pi.max_iter = q.max_iter;
        int st = check_common(q.dirty, q.ny, q.nx, q.psf, q.psf_ny, q.psf_nx, &pi, q.residual, q.comp_idx,
                              q.comp_flux, q.comp_cap);
        if (st) return fail(st, "problem %d: %s", i, g_last_error.c_str());
        const int ty = q.tiles_y > 0 ? q.tiles_y : 1, tx = q.tiles_x > 0 ? q.tiles_x : 1;
        if (q.tiles_y < 0 || q.tiles_x < 0 || ty > q.ny || tx > q.nx)
            return fail(CLEAN_E_INVAL, "problem %d: tile grid %d x %d for a %d x %d image", i, q.tiles_y, q.tiles_x,
                        q.ny, q.nx);
        if ((int64_t)ty * tx > MAX_TILES)
            return fail(CLEAN_E_UNSUPPORTED, "problem %d: %d tiles exceed %d", i, ty * tx, MAX_TILES);
        pty[i] = ty;
        ptx[i] = tx;
        if (ty * tx > 1) {
            if (q.interval < 1 || q.interval > MAX_INTERVAL)
                return fail(CLEAN_E_INVAL, "problem %d: feedback interval %d not in [1, %d]", i, q.interval,
                            MAX_INTERVAL);
            const int64_t smallest = (int64_t)(q.ny / ty) * (q.nx / tx);
            const double worst = (double)ty * tx * q.interval * (double)((int64_t)q.ny * q.nx - smallest) *
                                 (half ? 2.0 : 4.0);
            if (worst > GATHER_MAX_BYTES)
                return fail(CLEAN_E_UNSUPPORTED, "problem %d: a round of direct-gather feedback could read %.3g bytes "
                            "of PSF, more than a round may take within the device's wait limit", i, worst);
            pint[i] = q.interval;
            max_interval = std::max(max_interval, q.interval);
            any_tiled = true;
        }
        for (int a = 0; a < ty; ++a)
            for (int b = 0; b < tx; ++b) {
                const int h = (int)((int64_t)(a + 1) * q.ny / ty - (int64_t)a * q.ny / ty);
                const int w = (int)((int64_t)(b + 1) * q.nx / tx - (int64_t)b * q.nx / tx);
                ptile[i] = std::max<int64_t>(ptile[i], (int64_t)h * w);
                if (w % 4) w4 = false;
            }
    }
    const int V = w4 ? 4 : 1;
    hipStream_t stream = (hipStream_t)stream_v;
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // dynamic LDS of the tiled variant: a tile leader's round list, or the
    // gather's staged components
    const size_t dyn_lds = any_tiled ? std::max((size_t)16 * ((max_interval + 3) & ~3), (size_t)8 * GATHER_CHUNK) : 0;
    // workgroups of problem i at pp pixels per thread: its tiles' clusters
    auto members_of = [&](int i, int pp) -> int64_t {
        return (int64_t)pty[i] * ptx[i] * ((ptile[i] + (int64_t)WG * pp - 1) / ((int64_t)WG * pp));
    };
    // grid size of a launch shape, and whether its clusters fit the per-XCD
    // schedule (the grid's share of each XCD holds the largest problem)
    auto plan = [&](int pp, int &max_wg_out, bool &xcd_out) -> int {
        BFn f = pick_batched(half, V, pp / V, any_tiled);
        if (!f) return CLEAN_E_UNSUPPORTED;
        if (dyn_lds > 48 * 1024)
            HIPCHK(hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
        int oc = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&oc, (const void *)f, WG, dyn_lds));
        oc = std::min(oc, MAX_WG_PER_CU);
        int64_t seats = 0, mcs = 0;
        for (int i = 0; i < n; ++i) {
            const int64_t c = members_of(i, pp);
            seats += c;
            mcs = std::max(mcs, c);
        }
        max_wg_out = oc * ncu;
        const int64_t w = std::min<int64_t>(max_wg_out, seats);
        xcd_out = w % 8 == 0 && mcs <= w / 8 && mcs < 4096;
        return CLEAN_OK;
    };
    int ppt = shared->px_per_thread;
    if (ppt == 0 && btune_lookup(dev, batch_signature(probs, n, shared), ppt) && !valid_ppt(V, ppt)) ppt = 0;
    if (ppt == 0) {
        // no tuned shape for this batch (clean_autotune_batched): the rule.
        // 32 pixels per thread when the per-XCD schedule takes it: two
        // workgroups per CU and exchanges inside one L2 (the fastest shape
        // on 256 images of 128^2..1024^2).  Else 64: half the workgroups per
        // problem, so twice as many problems run at once across the device
        // (faster there than 32 px/thread across the device).
        ppt = V == 4 ? 64 : 16;
        int mw = 0;
        bool xok = false;
        if (V == 4 && plan(32, mw, xok) == CLEAN_OK && xok) ppt = 32;
    }
    if (!valid_ppt(V, ppt)) return fail(CLEAN_E_INVAL, "px_per_thread %d not available", ppt);
    const int K = ppt / V;
    BFn fn = pick_batched(half, V, K, any_tiled);
    if (!fn) return fail(CLEAN_E_UNSUPPORTED, "no batched kernel for %d x %d pixels per thread", K, V);
    if (dyn_lds > 48 * 1024)
        HIPCHK(hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds));
    int occ = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)fn, WG, dyn_lds));
    occ = std::min(occ, MAX_WG_PER_CU);
    const int max_wg = occ * ncu;

    // cluster size per problem (per tile for tiled ones), workgroups per
    // problem, then most workgroups first (largest images first among equals)
    std::vector<int> cs(n), mem(n);
    for (int i = 0; i < n; ++i) {
        cs[i] = (int)((ptile[i] + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
        const int64_t m = members_of(i, ppt);
        if (m > max_wg || m > 4095)
            return fail(CLEAN_E_UNSUPPORTED, "problem %d needs %lld workgroups, only %d fit", i, (long long)m,
                        std::min(max_wg, 4095));
        mem[i] = (int)m;
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (mem[x] != mem[y]) return mem[x] > mem[y];
        const int64_t px = (int64_t)probs[x].ny * probs[x].nx, py = (int64_t)probs[y].ny * probs[y].nx;
        return px > py;
    });

    // workspace: header (cleared) | jobs | tiled descriptions | seat0 |
    // partials | tiled round lists and feedback buffers | ticket table
    std::vector<int32_t> seat0(n + 1, 0);
    size_t nslots = 0, npart = 0, ntile_words = 0, nlist = 0, nacc = 0, nctl = 0;
    int ntiled = 0;
    for (int r = 0; r < n; ++r) {
        const int i = order[r];
        const int T = pty[i] * ptx[i];
        seat0[r + 1] = seat0[r] + mem[i];
        nslots += (size_t)T * 2 * ((cs[i] + 31) / 32 * 32);
        npart += mem[i];
        if (T > 1) {
            ++ntiled;
            ntile_words += align_up((size_t)T * 16, 256);                       // tile keys, round counts
            nlist += 4 * align_up((size_t)T * pint[i] * 4, 256);
            nacc += align_up((size_t)probs[i].ny * probs[i].nx * 4, 256);
            nctl += 256;                                                        // barrier counter, cancel word
        }
    }
    size_t o = 0;
    const size_t o_ctl = o;   o = align_up(o + sizeof(DevCtl), 256);
    const size_t o_stat = o;  o = align_up(o + sizeof(DevStat) * n, 256);
    const size_t o_slots = o; o = align_up(o + nslots * 8, 256);
    const size_t o_xq = o;    o = align_up(o + sizeof(XcdQueue), 256);
    const size_t o_tctl = o;  o = align_up(o + nctl, 256);
    const size_t o_twords = o; o = align_up(o + ntile_words, 256);
    const size_t head_end = o;
    const size_t o_lslots = o; o = align_up(o + nslots * 8, 256);
    const size_t o_jobs = o;  o = align_up(o + sizeof(PlainJob) * n, 256);
    const size_t o_tjobs = o; o = align_up(o + sizeof(KArgs) * ntiled, 256);
    const size_t o_tof = o;   o = align_up(o + sizeof(int32_t) * n, 256);
    const size_t o_seat = o;  o = align_up(o + sizeof(int32_t) * (n + 1), 256);
    const size_t o_part = o;  o = align_up(o + npart * 8, 256);
    const size_t o_lists = o; o = align_up(o + nlist, 256);
    const size_t o_acc = o;   o = align_up(o + nacc, 256);
    // per-XCD schedule when each XCD's share of the grid can hold the largest
    // problem (the kernel checks the actual placement before using it); its
    // ticket table only then
    const int W = std::min(max_wg, seat0[n]);
    const int max_cs = *std::max_element(mem.begin(), mem.end());
    const bool xcd_mode = W % 8 == 0 && max_cs <= W / 8 && max_cs < 4096;
    const size_t o_xtab = o;
    o = align_up(o + (xcd_mode ? (size_t)XQ_N * seat0[n] * sizeof(int32_t) : 0), 256);
    void *wp = nullptr;
    int st = internal_workspace(dev, o, &wp);
    if (st) return st;
    char *ws = (char *)wp;

    uint64_t ticks = 0;
    st = device_timeout_ticks(dev, ticks);
    if (st) return st;
    std::vector<PlainJob> jobs(n);
    std::vector<int32_t> tiled_of(n, -1);
    std::vector<KArgs> tjobs;
    tjobs.reserve(ntiled);
    size_t so = 0, po = 0, two = 0, lo = 0, ao = 0, co = 0;
    for (int r = 0; r < n; ++r) {
        const int i = order[r];
        const clean_problem &q = probs[i];
        const int T = pty[i] * ptx[i];
        const int pad = (cs[i] + 31) / 32 * 32;
        PlainJob &j = jobs[r];
        j.dirty = q.dirty; j.residual = q.residual; j.model = q.model;
        j.psf = q.psf; j.psf_bytes = (uint64_t)q.psf_ny * q.psf_nx * (half ? 2 : 4);
        j.ny = q.ny; j.nx = q.nx; j.psf_nx = q.psf_nx; j.cy = q.psf_ny / 2; j.cx = q.psf_nx / 2;
        j.cs = mem[i];               // workgroups of the problem (plain: its cluster)
        j.slot_pad = pad;
        j.gain = (float)shared->gain;
        j.threshold = q.threshold;
        j.max_iter = q.max_iter;
        j.cap = q.comp_cap;
        j.comp_idx = q.comp_idx; j.comp_flux = q.comp_flux;
        j.slots = (uint64_t *)(ws + o_slots) + so;
        j.lslots = (uint64_t *)(ws + o_lslots) + so;
        j.dstat = (DevStat *)(ws + o_stat) + r;
        j.partial = (double *)(ws + o_part) + po;
        tiled_of[r] = -1;
        if (T > 1) {
            KArgs a{};
            a.dirty = q.dirty; a.residual = q.residual; a.model = q.model;
            a.psf = q.psf; a.psf_bytes = j.psf_bytes;
            a.ny = q.ny; a.nx = q.nx; a.psf_ny = q.psf_ny; a.psf_nx = q.psf_nx;
            a.cy = q.psf_ny / 2; a.cx = q.psf_nx / 2;
            a.ty = pty[i]; a.tx = ptx[i]; a.T = T;
            a.cs = cs[i];
            a.ncl = T;
            a.slot_pad = pad;
            a.interval = pint[i];
            a.level_frac = shared->feedback_level;
            a.gather_parts = std::max(1, mem[i] / T);
            a.gain = (float)shared->gain;
            a.threshold = q.threshold;
            a.max_iter = q.max_iter;
            a.cap = q.comp_cap;
            a.timeout_ticks = ticks;
            a.comp_idx = q.comp_idx;
            a.comp_flux = q.comp_flux;
            a.cancel = (const int32_t *)shared->cancel;
            a.has_cancel = shared->cancel != nullptr;
            a.ctl = (DevCtl *)(ws + o_ctl);
            a.bar = (uint32_t *)(ws + o_tctl + co);
            a.cword = (uint32_t *)(ws + o_tctl + co + 128);
            a.dstat = j.dstat;
            a.role = nullptr;
            a.xslots = j.slots;
            a.lslots = j.lslots;
            char *tw = ws + o_twords + two;
            a.tile_key = (uint64_t *)tw;
            a.rb_n = (int32_t *)(tw + (size_t)T * 8);
            a.ag_n = (int32_t *)(tw + (size_t)T * 12);
            const size_t lb = align_up((size_t)T * pint[i] * 4, 256);
            a.rb_idx = (int32_t *)(ws + o_lists + lo);
            a.rb_flux = (float *)(ws + o_lists + lo + lb);
            a.ag_pos = (int32_t *)(ws + o_lists + lo + 2 * lb);
            a.ag_flux = (float *)(ws + o_lists + lo + 3 * lb);
            a.accbuf = (float *)(ws + o_acc + ao);
            a.partial = j.partial;
            a.hslots = nullptr;
            a.hpad = 0;
            tiled_of[r] = (int)tjobs.size();
            tjobs.push_back(a);
            two += align_up((size_t)T * 16, 256);
            lo += 4 * lb;
            ao += align_up((size_t)q.ny * q.nx * 4, 256);
            co += 256;
        }
        so += (size_t)T * 2 * pad;
        po += mem[i];
    }
    BatchArgs b{};
    b.jobs = (const PlainJob *)(ws + o_jobs);
    b.seat0 = (const int32_t *)(ws + o_seat);
    b.n = n;
    b.ctl = (DevCtl *)(ws + o_ctl);
    b.timeout_ticks = ticks;
    b.xcd_mode = xcd_mode;
    b.max_cs = max_cs;
    b.tickets = seat0[n];
    b.xq = (XcdQueue *)(ws + o_xq);
    b.xtable = (int32_t *)(ws + o_xtab);
    b.tjobs = (const KArgs *)(ws + o_tjobs);
    b.tiled_of = (const int32_t *)(ws + o_tof);
    b.cancel = (const int32_t *)shared->cancel;
    HIPCHK(hipMemsetAsync(ws, 0, head_end, stream));
    HIPCHK(hipMemcpyAsync(ws + o_jobs, jobs.data(), sizeof(PlainJob) * n, hipMemcpyHostToDevice, stream));
    if (ntiled)
        HIPCHK(hipMemcpyAsync(ws + o_tjobs, tjobs.data(), sizeof(KArgs) * ntiled, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + o_tof, tiled_of.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(ws + o_seat, seat0.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, stream));
    if (shared->flags & CLEAN_FLAG_CHECK_FINITE) {
        uint32_t *flag = &b.ctl->finite_bad;
        for (int i = 0; i < n; ++i) {
            const clean_problem &q = probs[i];
            hipLaunchKernelGGL(finite_check_kernel, dim3(256), dim3(256), 0, stream, q.dirty, (int64_t)q.ny * q.nx, flag);
            if (half)
                hipLaunchKernelGGL(finite_check_half_kernel, dim3(256), dim3(256), 0, stream,
                                   (const unsigned short *)q.psf, (int64_t)q.psf_ny * q.psf_nx, flag);
            else
                hipLaunchKernelGGL(finite_check_kernel, dim3(256), dim3(256), 0, stream, (const float *)q.psf,
                                   (int64_t)q.psf_ny * q.psf_nx, flag);
        }
        HIPCHK(hipGetLastError());
        uint32_t bad = 0;
        const D2H rb[1] = {{&bad, flag, 4}};
        st = read_back(rb, 1, stream);
        if (st) return st;
        if (bad) return fail(CLEAN_E_NONFINITE, "non-finite value in a dirty image or PSF");
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, stream));
    void *args[] = {(void *)&b};
    hipError_t le = hipLaunchCooperativeKernel((const void *)fn, dim3(W), dim3(WG), args, (unsigned)dyn_lds, stream);
    if (le != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(CLEAN_E_HIP, "cooperative launch of %d x %d failed: %s", W, WG, hipGetErrorString(le));
    }
    HIPCHK(hipEventRecord(e1, stream));
    hipLaunchKernelGGL(finalize_batch_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, b.jobs, n);
    HIPCHK(hipGetLastError());
    std::vector<DevStat> ds(n);
    DevCtl ctl{};
    const D2H rb[2] = {{ds.data(), ws + o_stat, sizeof(DevStat) * n}, {&ctl, b.ctl, sizeof ctl}};
    st = read_back(rb, 2, stream);
    if (st) return st;
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ctl.abort & ABORT_TIMEOUT) return fail(CLEAN_E_TIMEOUT, "a device-side wait timed out");
    if (ctl.abort) return fail(CLEAN_E_HIP, "device abort code %u", ctl.abort);
    if (stats) {
        for (int r = 0; r < n; ++r) {
            const int i = order[r];
            clean_stats &s = stats[i];
            memset(&s, 0, sizeof s);
            s.n_iter = ds[r].n_iter;
            s.stop_reason = ds[r].stop;
            s.n_rounds = ds[r].n_rounds;
            s.final_peak = ds[r].final_peak;
            s.residual_rms = std::sqrt(ds[r].sumsq / ((double)probs[i].ny * probs[i].nx));
            s.model_flux = ds[r].model_flux;
            s.device_ms = ms;
            s.wg_per_tile = cs[i];                 // per tile for tiled problems
            s.px_per_thread = ppt;
            s.workgroups = W;
            s.streamed = 0;
            s.xcd_local_clusters = ds[r].xcd_local;
            s.exchange_levels = 1;
        }
    }
    return CLEAN_OK;
}

int clean_autotune_batched(const clean_problem *probs, int n, const clean_params *shared, int64_t trial_iter,
                           int *px_per_thread, float *trial_ms, void *stream)
{
    g_last_error.clear();
    if (!probs || !shared || !px_per_thread) return fail(CLEAN_E_INVAL, "probs, shared and px_per_thread must be non-NULL");
    if (n < 1 || n > 65536) return fail(CLEAN_E_INVAL, "batch of %d problems not in [1, 65536]", n);
    if (trial_iter < 1) return fail(CLEAN_E_INVAL, "trial_iter must be >= 1");
    *px_per_thread = 0;
    static const int cand[CLEAN_BATCH_TUNE_CANDIDATES] = {8, 16, 32, 64};
    if (trial_ms)
        for (int c = 0; c < CLEAN_BATCH_TUNE_CANDIDATES; ++c) trial_ms[c] = -1.f;
    // trial copies: each problem capped at trial_iter iterations
    std::vector<clean_problem> trial(probs, probs + n);
    for (auto &q : trial) q.max_iter = std::min<int64_t>(q.max_iter, trial_iter);
    std::vector<clean_stats> st(n);
    clean_params sp = *shared;
    float best_ms = -1.f;
    int best = 0;
    const int V = batch_group_width(probs, n);
    for (int c = 0; c < CLEAN_BATCH_TUNE_CANDIDATES; ++c) {
        if (!valid_ppt(V, cand[c])) continue;
        sp.px_per_thread = cand[c];
        const int rc = clean_batched(trial.data(), n, &sp, st.data(), stream);
        if (rc == CLEAN_E_UNSUPPORTED) continue;   // shape does not fit this batch
        if (rc) return rc;                         // argument errors as clean_batched's
        if (trial_ms) trial_ms[c] = st[0].device_ms;
        if (best_ms < 0 || st[0].device_ms < best_ms) {
            best_ms = st[0].device_ms;
            best = cand[c];
        }
    }
    g_last_error.clear();
    if (best_ms < 0) return fail(CLEAN_E_UNSUPPORTED, "no candidate launch shape fits this batch");
    *px_per_thread = best;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_btune_mu);
    g_btune_cache[{dev, batch_signature(probs, n, shared)}] = best;
    return CLEAN_OK;
}

size_t clean_workspace_size(int ny, int nx, int tiles_y, int tiles_x, int feedback_interval, const clean_params *p)
{
    if (!p || ny <= 0 || nx <= 0 || tiles_y < 1 || tiles_x < 1 || tiles_y > ny || tiles_x > nx) return 0;
    const bool tiled = !(tiles_y == 1 && tiles_x == 1);
    const int T = tiles_y * tiles_x;
    if (T > MAX_TILES) return 0;
    if (tiled && (feedback_interval < 1 || feedback_interval > MAX_INTERVAL)) return 0;
    // an upper bound over the launch shapes the library may pick
    const int64_t npix = (int64_t)ny * nx;
    const int cs_max = 4096;
    const int W_max = 8192;
    FftGeom fg;
    if (tiled && (p->flags & CLEAN_FLAG_FFT_FEEDBACK)) {
        g_last_error.clear();
        if (fft_geometry(ny, nx, p->flags, fg) != CLEAN_OK) return 0;
    }
    const Layout L = make_layout(T, tiled ? cs_max / T + 64 : cs_max, (cs_max + 31) / 32 * 32,
                                 tiled ? feedback_interval : 1, W_max, npix, tiled, ny, fg);
    return L.total;
}

namespace {
using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;   // dev, ny, nx, ty, tx, dtype, stream flag, interval
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune_cache;
}

int clean_autotune(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx, int tiles_y,
                   int tiles_x, int feedback_interval, const clean_params *p, float *residual, int32_t *comp_idx,
                   float *comp_flux, int64_t comp_cap, int64_t trial_iter, clean_params *best, void *stream)
{
    g_last_error.clear();
    if (!best || !p) return fail(CLEAN_E_INVAL, "params and best must be non-NULL");
    const bool tiled = !(tiles_y == 1 && tiles_x == 1);
    if (trial_iter < 1) return fail(CLEAN_E_INVAL, "trial_iter must be >= 1");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const TuneKey key{dev, ny, nx, tiles_y, tiles_x, p->psf_dtype, p->flags & CLEAN_FLAG_STREAM_RESIDUAL,
                      tiled ? feedback_interval : 0};
    *best = *p;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            best->wg_per_tile = it->second.first;
            best->px_per_thread = it->second.second;
            return CLEAN_OK;
        }
    }
    // candidate shapes: each pixels-per-thread option with the smallest
    // cluster that holds the largest tile, and with twice that many workgroups
    int64_t max_tile = 0;
    bool w4 = true;
    for (int i = 0; i < tiles_y; ++i)
        for (int j = 0; j < tiles_x; ++j) {
            const int h = (int)((int64_t)(i + 1) * ny / tiles_y - (int64_t)i * ny / tiles_y);
            const int w = (int)((int64_t)(j + 1) * nx / tiles_x - (int64_t)j * nx / tiles_x);
            max_tile = std::max<int64_t>(max_tile, (int64_t)h * w);
            if (w % 4) w4 = false;
        }
    std::vector<int> ppts = w4 ? std::vector<int>{8, 16, 32, 64} : std::vector<int>{4, 16, 32};
    clean_params trial = *p;
    trial.max_iter = std::min<int64_t>(trial_iter, p->max_iter);
    const int64_t cap = std::min<int64_t>(comp_cap, trial.max_iter);
    float best_ms = -1.f;
    int best_cs = 0, best_ppt = 0;
    for (int ppt : ppts) {
        if (tiled && ppt > 32) continue;
        const int cs0 = (int)((max_tile + (int64_t)WG * ppt - 1) / ((int64_t)WG * ppt));
        for (int mult = 1; mult <= 2; ++mult) {
            trial.wg_per_tile = cs0 * mult;
            trial.px_per_thread = ppt;
            clean_stats st{};
            const int rc = tiled ? run(true, dirty, ny, nx, psf, psf_ny, psf_nx, tiles_y, tiles_x, feedback_interval,
                                       &trial, residual, comp_idx, comp_flux, cap, nullptr, nullptr, 0, &st, stream)
                                 : run(false, dirty, ny, nx, psf, psf_ny, psf_nx, 1, 1, 1, &trial, residual, comp_idx,
                                       comp_flux, cap, nullptr, nullptr, 0, &st, stream);
            if (rc == CLEAN_E_INVAL || rc == CLEAN_E_UNSUPPORTED) continue;   // shape does not fit
            if (rc) return rc;
            if (best_ms < 0 || st.device_ms < best_ms) {
                best_ms = st.device_ms;
                best_cs = trial.wg_per_tile;
                best_ppt = ppt;
            }
        }
    }
    g_last_error.clear();
    if (best_ms < 0) return fail(CLEAN_E_UNSUPPORTED, "no candidate launch shape fits");
    best->wg_per_tile = best_cs;
    best->px_per_thread = best_ppt;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = {best_cs, best_ppt};
    return CLEAN_OK;
}

int clean_autotune_interval(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                            int tiles_y, int tiles_x, const int *candidates, int n_candidates,
                            const clean_params *p, int64_t trial_iter, double growth_limit, float *residual,
                            int32_t *comp_idx, float *comp_flux, int64_t comp_cap, int *interval,
                            double *rate_out, double *peak_ratio_out, void *stream)
{
    g_last_error.clear();
    if (!p || !interval) return fail(CLEAN_E_INVAL, "params and interval must be non-NULL");
    if (!candidates || n_candidates < 1 || n_candidates > 64)
        return fail(CLEAN_E_INVAL, "need 1..64 candidate intervals");
    for (int i = 0; i < n_candidates; ++i)
        if (candidates[i] < 1 || candidates[i] > MAX_INTERVAL)
            return fail(CLEAN_E_INVAL, "candidate interval %d not in [1, %d]", candidates[i], MAX_INTERVAL);
    if (tiles_y == 1 && tiles_x == 1) return fail(CLEAN_E_INVAL, "the interval only matters for a tile grid");
    if (trial_iter < 1) return fail(CLEAN_E_INVAL, "trial_iter must be >= 1");
    if (!(growth_limit > 0.0)) return fail(CLEAN_E_INVAL, "growth_limit must be > 0");
    *interval = 0;
    // the dirty image's peak: a run of no iterations
    clean_params trial = *p;
    trial.max_iter = 0;
    clean_stats st0{};
    int rc = run(true, dirty, ny, nx, psf, psf_ny, psf_nx, tiles_y, tiles_x, candidates[0], &trial, residual,
                 comp_idx, comp_flux, comp_cap, nullptr, nullptr, 0, &st0, stream);
    if (rc) return rc;
    const double peak0 = std::fabs(st0.final_peak);
    trial.max_iter = std::min<int64_t>(trial_iter, p->max_iter);
    const int64_t cap = std::min<int64_t>(comp_cap, trial.max_iter);
    double best_rate = -1.0;
    for (int i = 0; i < n_candidates; ++i) {
        clean_stats st{};
        rc = run(true, dirty, ny, nx, psf, psf_ny, psf_nx, tiles_y, tiles_x, candidates[i], &trial, residual, comp_idx,
                 comp_flux, cap, nullptr, nullptr, 0, &st, stream);
        if (rc) return rc;
        const double ratio = peak0 > 0.0 ? std::fabs(st.final_peak) / peak0 : (st.final_peak == 0.0 ? 0.0 : INFINITY);
        const double rate = st.device_ms > 0.f ? (double)st.n_iter / (st.device_ms * 1e-3) : 0.0;
        if (rate_out) rate_out[i] = rate;
        if (peak_ratio_out) peak_ratio_out[i] = ratio;
        const bool ok = std::isfinite(ratio) && std::isfinite(st.residual_rms) && ratio <= growth_limit;
        if (ok && rate > best_rate) {
            best_rate = rate;
            *interval = candidates[i];
        }
    }
    return CLEAN_OK;
}

int clean_beam_fit(const void *psf, int psf_ny, int psf_nx, int psf_dtype, int64_t *area, double *sigma,
                   void *stream_v)
{
    g_last_error.clear();
    if (!psf || !area || !sigma) return fail(CLEAN_E_INVAL, "psf, area and sigma must be non-NULL");
    if (psf_ny < 1 || psf_nx < 1) return fail(CLEAN_E_INVAL, "PSF size %d x %d", psf_ny, psf_nx);
    if (psf_dtype != CLEAN_PSF_F32 && psf_dtype != CLEAN_PSF_F16) return fail(CLEAN_E_INVAL, "psf_dtype %d", psf_dtype);
    hipStream_t stream = (hipStream_t)stream_v;
    const size_t es = psf_dtype == CLEAN_PSF_F16 ? 2 : 4;
    const int cy = psf_ny / 2, cx = psf_nx / 2;
    // a crop about the centre, doubled until the lobe does not reach its edge
    for (int half = 32;; half *= 2) {
        const int y0 = std::max(0, cy - half), y1 = std::min(psf_ny, cy + half);
        const int x0 = std::max(0, cx - half), x1 = std::min(psf_nx, cx + half);
        const int h = y1 - y0, w = x1 - x0;
        // staged through pinned host memory: an asynchronous copy into it is
        // complete once the stream is synchronised
        unsigned char *raw = nullptr;
        HIPCHK(hipHostMalloc((void **)&raw, (size_t)h * w * es, hipHostMallocDefault));
        std::vector<float> v((size_t)h * w);
        hipError_t ce = hipMemcpy2DAsync(raw, (size_t)w * es, (const char *)psf + ((size_t)y0 * psf_nx + x0) * es,
                                         (size_t)psf_nx * es, (size_t)w * es, h, hipMemcpyDeviceToHost, stream);
        if (ce == hipSuccess) ce = hipStreamSynchronize(stream);
        if (ce == hipSuccess)
            for (size_t i = 0; i < v.size(); ++i) {
                if (es == 4) {
                    std::memcpy(&v[i], &raw[i * 4], 4);
                } else {
                    __half hv;
                    std::memcpy(&hv, &raw[i * 2], 2);
                    v[i] = __half2float(hv);
                }
            }
        (void)hipHostFree(raw);
        if (ce != hipSuccess) return fail(CLEAN_E_HIP, "PSF crop copy: %s", hipGetErrorString(ce));
        const int c = (cy - y0) * w + (cx - x0);
        if (!(v[c] > 0.5f)) return fail(CLEAN_E_INVAL, "PSF centre value %g is not above one half", (double)v[c]);
        std::vector<unsigned char> seen(v.size(), 0);
        std::vector<int> queue;
        queue.reserve(1024);
        queue.push_back(c);
        seen[c] = 1;
        bool edge = false;
        for (size_t head = 0; head < queue.size(); ++head) {
            const int q = queue[head], y = q / w, x = q % w;
            if (y == 0 || x == 0 || y == h - 1 || x == w - 1) edge = true;
            const int yy[4] = {y - 1, y + 1, y, y}, xx[4] = {x, x, x - 1, x + 1};
            for (int k = 0; k < 4; ++k) {
                if (yy[k] < 0 || yy[k] >= h || xx[k] < 0 || xx[k] >= w) continue;
                const int r = yy[k] * w + xx[k];
                if (!seen[r] && v[r] > 0.5f) {
                    seen[r] = 1;
                    queue.push_back(r);
                }
            }
        }
        const bool whole = y0 == 0 && x0 == 0 && y1 == psf_ny && x1 == psf_nx;
        if (edge && !whole) continue;            // the lobe may go on past the crop
        *area = (int64_t)queue.size();
        *sigma = 2.0 * std::sqrt((double)*area / M_PI) / (2.0 * std::sqrt(2.0 * std::log(2.0)));
        return CLEAN_OK;
    }
}

int clean_restore(const double *model, const float *residual, int ny, int nx, double sigma, double *out,
                  void *stream_v)
{
    g_last_error.clear();
    if (!model || !residual || !out) return fail(CLEAN_E_INVAL, "model, residual and out must be non-NULL");
    if (ny < 1 || nx < 1) return fail(CLEAN_E_INVAL, "image size %d x %d", ny, nx);
    if (!(sigma > 0.0 && sigma <= 1000.0)) return fail(CLEAN_E_INVAL, "sigma %g not in (0, 1000]", sigma);
    if ((int64_t)ny * nx > ((int64_t)1 << 31)) return fail(CLEAN_E_UNSUPPORTED, "image larger than 2^31 pixels");
    hipStream_t stream = (hipStream_t)stream_v;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const int R = (int)std::ceil(5.0 * sigma);
    const int64_t npix = (int64_t)ny * nx;
    const size_t taps = align_up((size_t)(2 * R + 1) * 8, 256);
    void *wp = nullptr;
    int st = internal_workspace(dev, taps + (size_t)npix * 8, &wp);
    if (st) return st;
    double *b = (double *)wp;
    double *tmp = (double *)((char *)wp + taps);
    std::vector<double> hb(2 * R + 1);
    for (int d = -R; d <= R; ++d) hb[d + R] = std::exp(-((double)d * d) / (2.0 * sigma * sigma));
    HIPCHK(hipMemcpyAsync(b, hb.data(), hb.size() * 8, hipMemcpyHostToDevice, stream));
    const int blocks = (int)std::min<int64_t>(8192, (npix + 255) / 256);
    hipLaunchKernelGGL(restore_rows_kernel, dim3(blocks), dim3(256), 0, stream, model, tmp, ny, nx, b, R);
    hipLaunchKernelGGL(restore_cols_kernel, dim3(blocks), dim3(256), 0, stream, tmp, residual, out, ny, nx, b, R);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return CLEAN_OK;
}

int clean_psf_to_f16(const float *psf, uint16_t *out, int64_t n, void *stream_v)
{
    g_last_error.clear();
    if (!psf || !out || n < 0) return fail(CLEAN_E_INVAL, "bad arguments");
    hipStream_t stream = (hipStream_t)stream_v;
    if (n == 0) return CLEAN_OK;
    hipLaunchKernelGGL(to_half_kernel, dim3(2048), dim3(256), 0, stream, psf, (unsigned short *)out, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    return CLEAN_OK;
}

int clean_bandwidth_probe(void *buf, size_t bytes, int mode, int reps, double *gbs, void *stream_v)
{
    g_last_error.clear();
    if (!buf || !gbs) return fail(CLEAN_E_INVAL, "buf and gbs must be non-NULL");
    if (bytes < 4096 || bytes % 32) return fail(CLEAN_E_INVAL, "bytes %zu: at least 4096 and a multiple of 32", bytes);
    if (mode != 0 && mode != 1) return fail(CLEAN_E_INVAL, "mode %d is not 0 (read) or 1 (copy)", mode);
    if (reps < 1 || reps > 100000) return fail(CLEAN_E_INVAL, "reps %d not in [1, 100000]", reps);
    hipStream_t stream = (hipStream_t)stream_v;
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    void *sink = nullptr;
    int st = internal_workspace(dev, 4096, &sink);
    if (st) return st;
    const int blocks = 8 * ncu;             // 2048 workgroups of 256 threads on 256 CUs
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, stream));
    if (mode == 0)
        hipLaunchKernelGGL(probe_read_kernel, dim3(blocks), dim3(256), 0, stream, (const float4 *)buf,
                           (int64_t)(bytes / 16), reps, (float *)sink);
    else
        hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks), dim3(256), 0, stream, (const float4 *)buf,
                           (float4 *)((char *)buf + bytes / 2), (int64_t)(bytes / 32), reps);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) le = hipEventRecord(e1, stream);
    if (le == hipSuccess) le = hipEventSynchronize(e1);
    float ms = 0.f;
    if (le == hipSuccess) le = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (le != hipSuccess) return fail(CLEAN_E_HIP, "bandwidth probe: %s", hipGetErrorString(le));
    *gbs = ms > 0.f ? (double)bytes * reps / (ms * 1e-3) / 1e9 : 0.0;
    return CLEAN_OK;
}

size_t clean_set_workspace_limit(size_t bytes)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    const size_t old = g_ws_limit;
    g_ws_limit = bytes;
    return old;
}

const char *clean_strerror(int status)
{
    switch (status) {
    case CLEAN_OK: return "ok";
    case CLEAN_E_INVAL: return "invalid argument";
    case CLEAN_E_NONFINITE: return "non-finite input";
    case CLEAN_E_NOMEM: return "out of device memory or workspace too small";
    case CLEAN_E_HIP: return "HIP runtime error";
    case CLEAN_E_TIMEOUT: return "device-side wait timed out";
    case CLEAN_E_UNSUPPORTED: return "unsupported shape or option";
    }
    return "unknown status";
}

const char *clean_last_error(void) { return g_last_error.c_str(); }

const char *clean_version(void) { return "cleanhip 0.1.0 (gfx950)"; }

} // extern "C"

// ------------------------------------------------------------ plan tuner --
namespace {

// Cached plans: one line per key, "key<TAB>ty tx interval wg ppt lo hi rate".
std::mutex g_plan_mu;

std::string plan_key(int dev, int ny, int nx, int psf_ny, int psf_nx, const clean_params *p, int64_t trial_iter,
                     const int *grids, int n_grids, const int *intervals, int n_intervals, double lo, double hi)
{
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char &ch : arch)
        if (ch == '\t' || ch == '\n') ch = ' ';
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s|%dx%d|%dx%d|d%d|f%d|g%.17g|t%.17g|m%lld|T%lld|L%.17g|b%.17g,%.17g", arch.c_str(),
                  ny, nx, psf_ny, psf_nx, p->psf_dtype, p->flags, p->gain, p->threshold, (long long)p->max_iter,
                  (long long)trial_iter, p->feedback_level, lo, hi);
    std::string k = buf;
    k += "|G";
    for (int i = 0; i < n_grids; ++i) k += std::to_string(grids[2 * i]) + "x" + std::to_string(grids[2 * i + 1]) + ",";
    k += "|I";
    for (int i = 0; i < n_intervals; ++i) k += std::to_string(intervals[i]) + ",";
    return k;
}

bool plan_lookup(const char *path, const std::string &key, clean_plan *plan)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[4096];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        if (key != line) continue;
        clean_plan q{};
        if (std::sscanf(tab + 1, "%d %d %d %d %d %lf %lf %lf", &q.tiles_y, &q.tiles_x, &q.interval, &q.wg_per_tile,
                        &q.px_per_thread, &q.band_min, &q.band_max, &q.iters_per_s) == 8) {
            q.from_cache = 1;
            *plan = q;
            found = true;          // the last line for a key wins
        }
    }
    std::fclose(f);
    return found;
}

int plan_store(const char *path, const std::string &key, const clean_plan &q)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return fail(CLEAN_E_INVAL, "cannot open plan cache %s for appending", path);
    std::fprintf(f, "%s\t%d %d %d %d %d %.17g %.17g %.17g\n", key.c_str(), q.tiles_y, q.tiles_x, q.interval,
                 q.wg_per_tile, q.px_per_thread, q.band_min, q.band_max, q.iters_per_s);
    std::fclose(f);
    return CLEAN_OK;
}

// Device buffers of the tuner, freed on every exit path.
struct DevBufs {
    std::vector<void *> p;
    ~DevBufs()
    {
        for (void *q : p) (void)hipFree(q);
    }
    int get(size_t bytes, void **out)
    {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CLEAN_E_NOMEM, "tuner buffer of %zu bytes", bytes);
        }
        p.push_back(q);
        *out = q;
        return CLEAN_OK;
    }
};

// Smallest and largest a[i] - b[i] (NaN if any difference is not finite).
int diff_range(const double *a, const double *b, int64_t n, double *part, int nblk, hipStream_t stream, double &lo,
               double &hi)
{
    hipLaunchKernelGGL(diff_range_kernel, dim3(nblk), dim3(256), 0, stream, a, b, n, part);
    HIPCHK(hipGetLastError());
    std::vector<double> h(2 * (size_t)nblk);
    const D2H rb[1] = {{h.data(), part, h.size() * 8}};
    int st = read_back(rb, 1, stream);
    if (st) return st;
    lo = INFINITY;
    hi = -INFINITY;
    for (int i = 0; i < nblk; ++i) {
        if (std::isnan(h[2 * i]) || std::isnan(h[2 * i + 1])) { lo = hi = NAN; return CLEAN_OK; }
        lo = std::min(lo, h[2 * i]);
        hi = std::max(hi, h[2 * i + 1]);
    }
    return CLEAN_OK;
}

} // namespace

extern "C" int clean_autotune_plan(const float *dirty, int ny, int nx, const void *psf, int psf_ny, int psf_nx,
                                   const int *grids, int n_grids, const int *intervals, int n_intervals,
                                   const clean_params *p, int64_t trial_iter, double band_min, double band_max,
                                   const char *cache_path, clean_plan *plan, double *band_out, double *rate_out,
                                   void *stream_v)
{
    g_last_error.clear();
    if (!dirty || !psf || !p || !plan || !grids || !intervals) return fail(CLEAN_E_INVAL, "NULL argument");
    if (n_grids < 1 || n_grids > 16 || n_intervals < 1 || n_intervals > 16)
        return fail(CLEAN_E_INVAL, "need 1..16 tile grids and 1..16 intervals");
    for (int i = 0; i < n_grids; ++i)
        if (grids[2 * i] < 1 || grids[2 * i + 1] < 1 || grids[2 * i] > ny || grids[2 * i + 1] > nx ||
            (grids[2 * i] == 1 && grids[2 * i + 1] == 1) || grids[2 * i] * grids[2 * i + 1] > MAX_TILES)
            return fail(CLEAN_E_INVAL, "tile grid %d x %d", grids[2 * i], grids[2 * i + 1]);
    for (int i = 0; i < n_intervals; ++i)
        if (intervals[i] < 1 || intervals[i] > MAX_INTERVAL) return fail(CLEAN_E_INVAL, "interval %d", intervals[i]);
    if (trial_iter < 1) return fail(CLEAN_E_INVAL, "trial_iter must be >= 1");
    if (!(band_min <= 0.0 && band_max >= 0.0)) return fail(CLEAN_E_INVAL, "the band must contain 0");
    int st = check_common(dirty, ny, nx, psf, psf_ny, psf_nx, p, (float *)dirty, nullptr, nullptr, 0);
    if (st) return st;
    hipStream_t stream = (hipStream_t)stream_v;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    const std::string key = plan_key(dev, ny, nx, psf_ny, psf_nx, p, trial_iter, grids, n_grids, intervals,
                                     n_intervals, band_min, band_max);
    *plan = clean_plan{};
    const int ncand = n_grids * n_intervals;
    for (int i = 0; i < ncand; ++i) {
        if (band_out) band_out[2 * i] = band_out[2 * i + 1] = NAN;
        if (rate_out) rate_out[i] = NAN;
    }
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        if (plan_lookup(cache_path, key, plan)) return CLEAN_OK;
    }
    // the clean beam and the restored plain image of trial_iter iterations
    int64_t area = 0;
    double sigma = 0.0;
    st = clean_beam_fit(psf, psf_ny, psf_nx, p->psf_dtype, &area, &sigma, stream_v);
    if (st) return st;
    const int64_t npix = (int64_t)ny * nx;
    const int64_t n_it = std::min<int64_t>(trial_iter, p->max_iter);
    const int nblk = 1024;
    DevBufs B;
    void *res = nullptr, *idx = nullptr, *flux = nullptr, *model = nullptr, *rest_p = nullptr, *rest_t = nullptr,
         *part = nullptr;
    if ((st = B.get((size_t)npix * 4, &res)) || (st = B.get((size_t)std::max<int64_t>(n_it, 1) * 4, &idx)) ||
        (st = B.get((size_t)std::max<int64_t>(n_it, 1) * 4, &flux)) || (st = B.get((size_t)npix * 8, &model)) ||
        (st = B.get((size_t)npix * 8, &rest_p)) || (st = B.get((size_t)npix * 8, &rest_t)) ||
        (st = B.get((size_t)nblk * 16, &part)))
        return st;
    clean_params trial = *p;
    trial.max_iter = n_it;
    trial.wg_per_tile = 0;
    trial.px_per_thread = 0;
    clean_stats sp{};
    st = run(false, dirty, ny, nx, psf, psf_ny, psf_nx, 1, 1, 1, &trial, (float *)res, (int32_t *)idx, (float *)flux,
             n_it, (double *)model, nullptr, 0, &sp, stream_v);
    if (st) return st;
    st = clean_restore((const double *)model, (const float *)res, ny, nx, sigma, (double *)rest_p, stream_v);
    if (st) return st;
    // every (grid, interval): the band of restored(tiled) - restored(plain)
    clean_plan best{};
    for (int gi = 0; gi < n_grids; ++gi)
        for (int ii = 0; ii < n_intervals; ++ii) {
            clean_stats s{};
            st = run(true, dirty, ny, nx, psf, psf_ny, psf_nx, grids[2 * gi], grids[2 * gi + 1], intervals[ii], &trial,
                     (float *)res, (int32_t *)idx, (float *)flux, n_it, (double *)model, nullptr, 0, &s, stream_v);
            if (st == CLEAN_E_UNSUPPORTED) continue;           // no launch for this grid
            if (st) return st;
            st = clean_restore((const double *)model, (const float *)res, ny, nx, sigma, (double *)rest_t, stream_v);
            if (st) return st;
            double lo = 0.0, hi = 0.0;
            st = diff_range((const double *)rest_t, (const double *)rest_p, npix, (double *)part, nblk, stream, lo, hi);
            if (st) return st;
            const double rate = s.device_ms > 0.f ? (double)s.n_iter / (s.device_ms * 1e-3) : 0.0;
            const int ci = gi * n_intervals + ii;
            if (band_out) { band_out[2 * ci] = lo; band_out[2 * ci + 1] = hi; }
            if (rate_out) rate_out[ci] = rate;
            const bool ok = std::isfinite(lo) && std::isfinite(hi) && lo >= band_min && hi <= band_max &&
                            s.stop_reason != CLEAN_STOP_NONFINITE;
            if (ok && rate > best.iters_per_s) {
                best.tiles_y = grids[2 * gi];
                best.tiles_x = grids[2 * gi + 1];
                best.interval = intervals[ii];
                best.wg_per_tile = s.wg_per_tile;
                best.px_per_thread = s.px_per_thread;
                best.band_min = lo;
                best.band_max = hi;
                best.iters_per_s = rate;
            }
        }
    g_last_error.clear();
    *plan = best;
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        st = plan_store(cache_path, key, best);
        if (st) return st;
    }
    return CLEAN_OK;
}
