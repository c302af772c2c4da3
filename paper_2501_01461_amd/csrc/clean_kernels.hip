// clean_kernels.hip -- gfx950 kernels for the Hogbom CLEAN minor loop and its
// tiled-with-feedback form (Wright, Adamek, Armour, arXiv 2501.01461,
// Sections 2 and 3).  Host entry points live in clean_api.hip.
//
// Design (one persistent, cooperatively launched kernel per call):
//  * The residual lives in VGPRs for the whole run (RegTile), or, when the
//    co-resident register file cannot hold it, in the caller's residual array,
//    streamed every iteration (StreamTile).  A tile (the whole image for plain
//    CLEAN) is owned by a cluster of `cs` workgroups; thread t of cluster rank
//    g owns K groups of V consecutive pixels, group k at tile-local flat index
//    ((k*cs + g)*WG + t)*V.  Only the peak key crosses workgroups.
//  * One minor iteration: every thread applies r = fma(-c, psf[q - p + ctr], r)
//    to its pixels and keeps its own largest |r| (lowest index on ties); a
//    wave/LDS reduction gives the workgroup's key; the cluster's keys are
//    exchanged through per-workgroup slots written and polled with agent-scope
//    relaxed atomics (no fences: nothing else crosses workgroups per iteration).
//  * Tiled rounds add three grid barriers: after the local loops (round lists
//    published), after the feedback gather (all workgroups, including helpers,
//    compute the cross-coupling sum for a share of the pixels into a float32
//    buffer), and after each cluster has applied it and re-found its peak.
//    The FFT form (a compile-time specialisation) replaces the gather by
//    transform phases with grid barriers of their own.
//  * The batched kernel deals many independent images to clusters from a
//    seat queue; each runs the same plain minor loop.
//  * Every wait is bounded: a wall-clock limit or an abort flag set by any
//    workgroup ends it, and the kernel then returns with an error code.
//
// Peak key (64 bits): |v| bits (31) << 33 | (0x0FFFFFFF - f) << 5 | sign << 4 |
// tag (4).  The unsigned max of keys is the largest |v|, then the lowest
// tile-local index f (row-major inside the tile, so the lowest image index);
// the tag marks which exchange a published key belongs to.  Every NaN enters
// the key as the one magnitude 0x7FC00000, above +Inf: a region holding a NaN
// has its lowest-index NaN as its peak.  A non-finite peak ends the run.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "clean_device.h"
#include "clean_fft.h"

namespace cleanhip {

// ------------------------------------------------------------ primitives --

__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The caller's cancel flag, a word of host memory (system scope: not cached).
__device__ __forceinline__ uint32_t host_flag(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0 ? 1u : 0u;
}

// A store that ends in this XCD's L2 (sc0: written through the CU's L1, not
// on to the point of coherence of all XCDs as a device-scope store is).  A
// device-scope load (ld_agent) from any CU of the same XCD misses its L1 and
// reads that L2, so it sees the value; one from another XCD may not.  Only
// workgroups known to share an XCD exchange data this way.  Measured round
// trip between two workgroups of one XCD: 0.46 us, against 0.81 us with
// device-scope stores.  (An sc0 load is no substitute for ld_agent here: it
// may be served by the reader's own L1 and never see the store.)
__device__ __forceinline__ void st_xcd(uint64_t *p, uint64_t v)
{
    asm volatile("global_store_dwordx2 %0, %1, off sc0" : : "v"(p), "v"(v) : "memory");
}

// The XCD (accelerator complex die) this wave runs on.
__device__ __forceinline__ uint32_t xcc_id()
{
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(x));
    return x & 15u;
}

// Data written by one workgroup and read by another inside the launch goes
// through agent-coherent accesses (write-through stores, loads that do not hit
// stale cache lines).  The grid barrier then only has to order them: every
// wave has waited for its stores before the workgroup arrives, and readers
// load after the barrier has released, so no cache write-back or invalidation
// is needed and the PSF stays cached across rounds.
// The pointers are cast to the global address space: generic (flat) accesses
// would also count against the LDS counter, so that every wait for an LDS
// access would wait for them as well.
template <typename T> __device__ __forceinline__ T ldc(const T *p)
{
    return __hip_atomic_load((__attribute__((address_space(1))) const T *)p, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ void stc(T *p, T v)
{
    __hip_atomic_store((__attribute__((address_space(1))) T *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// |v| as the peak search orders it: IEEE magnitude bits (+Inf above every
// finite value), every NaN given the quiet NaN's magnitude, above +Inf.
__device__ __forceinline__ uint32_t peak_mag(uint32_t bits)
{
    const uint32_t m = bits & 0x7FFFFFFFu;
    return m > 0x7F800000u ? 0x7FC00000u : m;
}
__device__ __forceinline__ uint64_t make_key(uint32_t bits, uint32_t f)
{
    return ((uint64_t)peak_mag(bits) << 33) | ((uint64_t)(0x0FFFFFFFu - f) << 5) |
           ((uint64_t)(bits >> 31) << 4);
}
// Largest |a|, |b| with NaN propagating (one v_maximum3_f32 for three values).
__device__ __forceinline__ float nan_max(float a, float b) { return __builtin_elementwise_maximum(a, b); }
__device__ __forceinline__ bool is_nan(float x) { return x != x; }
__device__ __forceinline__ float key_value(uint64_t k)
{
    uint32_t a = (uint32_t)(k >> 33);
    uint32_t s = (uint32_t)(k >> 4) & 1u;
    return __uint_as_float(a | (s << 31));
}
__device__ __forceinline__ uint32_t key_f(uint64_t k)
{
    return 0x0FFFFFFFu - (uint32_t)((k >> 5) & 0x0FFFFFFFu);
}
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// One DPP step of a 64-bit max: take the (row-shifted or row-broadcast)
// neighbour's key when it is larger; lanes without a source read 0.
#define CLEAN_DPP_MAX_STEP(k, CTRL, ROW_MASK)                                                          \
    do {                                                                                              \
        const uint32_t plo_ = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(k), CTRL, ROW_MASK, 0xf, true); \
        const uint32_t phi_ = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)((k) >> 32), CTRL, ROW_MASK, 0xf, true); \
        const uint64_t p_ = ((uint64_t)phi_ << 32) | plo_;                                            \
        k = p_ > (k) ? p_ : (k);                                                                      \
    } while (0)

// Max of a 64-bit key over the wave, uniform on return: row_shr 1/2/4/8 leaves
// each row's maximum in its lane 15, row_bcast 15/31 carries them up to lane 63.
__device__ __forceinline__ uint64_t wave_max64(uint64_t k)
{
    CLEAN_DPP_MAX_STEP(k, 0x111, 0xf);   // row_shr:1
    CLEAN_DPP_MAX_STEP(k, 0x112, 0xf);   // row_shr:2
    CLEAN_DPP_MAX_STEP(k, 0x114, 0xf);   // row_shr:4
    CLEAN_DPP_MAX_STEP(k, 0x118, 0xf);   // row_shr:8
    CLEAN_DPP_MAX_STEP(k, 0x142, 0xa);   // row_bcast:15 into rows 1 and 3
    CLEAN_DPP_MAX_STEP(k, 0x143, 0xc);   // row_bcast:31 into rows 2 and 3
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)k, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(k >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double wave_sum64f(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Raw buffer resource over [base, base + bytes): loads past the end return 0
// instead of touching memory, a guard behind the host's shape checks.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint64_t bytes)
{
    uint32_t n = bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n, 0x00020000);
}

// The same for a base and size that are equal in all lanes of the wave (one
// PSF window per wave) where the compiler cannot prove it (inside a
// non-inlined function, or when the window comes from memory): both go to
// scalar registers.  Without that the compiler wraps each load in a loop over
// the wave's distinct descriptors and waits for every load before the next.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_uniform(const void *base, uint64_t bytes)
{
    const uint32_t n = __builtin_amdgcn_readfirstlane(bytes > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)bytes);
    const uint64_t p = (uint64_t)(uintptr_t)base;
    const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(p >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)p);
    return __builtin_amdgcn_make_buffer_rsrc((void *)(uintptr_t)u, (short)0, (int)n, 0x00020000);
}

// min(max(x, 0), 2^32 - 1) for a 64-bit x, with 32-bit compares only: the
// scalar unit has no 64-bit ordered compare, so a 64-bit one would move the
// whole computation to the vector unit.
__device__ __forceinline__ uint32_t clamp_u32(int64_t x)
{
    const int32_t hi = (int32_t)((uint64_t)x >> 32);
    return hi < 0 ? 0u : hi > 0 ? 0xFFFFFFFFu : (uint32_t)x;
}

// A value that is equal in all lanes of the wave, moved to scalar registers
// (each 32-bit word from the first active lane), for code where the compiler
// cannot prove it uniform: function arguments and loads through them.
template <typename T> __device__ __forceinline__ T wave_uniform(const T &v)
{
    static_assert(sizeof(T) % 4 == 0, "whole 32-bit words");
    uint32_t w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// V consecutive PSF values, widened to float, at byte offset `off`.
template <typename PT, int V> struct PsfLoad;
template <> struct PsfLoad<float, 4> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, float *o)
    {
        load_s(rs, off, 0, o);
    }
    // voffset plus a uniform (scalar) offset
    static __device__ __forceinline__ void load_s(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, float *o)
    {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0);
        o[0] = __uint_as_float(v[0]); o[1] = __uint_as_float(v[1]);
        o[2] = __uint_as_float(v[2]); o[3] = __uint_as_float(v[3]);
    }
};
template <> struct PsfLoad<float, 1> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, float *o)
    {
        o[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
    }
};
template <> struct PsfLoad<__half, 4> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, float *o)
    {
        load_s(rs, off, 0, o);
    }
    static __device__ __forceinline__ void load_s(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, float *o)
    {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
        o[0] = __half2float(__ushort_as_half((unsigned short)(v[0] & 0xFFFFu)));
        o[1] = __half2float(__ushort_as_half((unsigned short)(v[0] >> 16)));
        o[2] = __half2float(__ushort_as_half((unsigned short)(v[1] & 0xFFFFu)));
        o[3] = __half2float(__ushort_as_half((unsigned short)(v[1] >> 16)));
    }
};
template <> struct PsfLoad<__half, 1> {
    static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, float *o)
    {
        o[0] = __half2float(__ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0)));
    }
};

// ------------------------------------------------------- abort & timing --

// Where waits look for an abort and how long they may last.
struct Sync {
    DevCtl *ctl;
    uint64_t timeout_ticks;
};

__device__ __forceinline__ bool aborted(const Sync &y)
{
    return ld_agent32(&y.ctl->abort) != 0;
}
__device__ __forceinline__ void raise_abort(const Sync &y, uint32_t code)
{
    __hip_atomic_fetch_or(&y.ctl->abort, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------ cluster reduction ------

// Cluster-wide max of the threads' keys for exchange number `e`.  A DPP wave
// max, then wave 0 takes the max of the waves' keys from LDS (every lane reads
// all of them: a short scalar-like chain, no second cross-lane pass),
// publishes the workgroup's key in its slot and polls the cluster's slots
// until every slot carries this exchange's tag.  When the cluster is known to
// share one XCD the slots are `lslots`, written with XCD-local stores, else
// `slots`, written with agent-scope relaxed atomics; both are polled with
// agent-scope loads.  Two workgroup
// barriers per call.  Returns false if the run was aborted; `out` is uniform
// on return.
__device__ bool cluster_reduce(const Sync &y, uint64_t *slots, uint64_t *lslots, int slot_pad, int cs, int rank,
                               uint32_t e, uint64_t tkey, uint64_t &out)
{
    __shared__ uint64_t s_wave[NWAVES];
    __shared__ uint64_t s_res;
    __shared__ int s_good;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t wk = wave_max64(tkey);
    if (lane == 0) s_wave[wave] = wk;
    __syncthreads();
    if (wave == 0) {
        uint64_t g = s_wave[0];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) g = umax64(g, s_wave[w]);
        bool ok = true;
        if (cs > 1) {
            const uint64_t tag = (uint64_t)((e & 7u) + 1u);
            const bool local = lslots != nullptr;
            uint64_t *blk = (local ? lslots : slots) + (size_t)(e & 1u) * slot_pad;
            if (lane == 0) {
                if (local) st_xcd(&blk[rank], (g & ~15ull) | tag);
                else st_agent(&blk[rank], (g & ~15ull) | tag);
            }
            const uint64_t t0 = wall_clock64();
            uint32_t spins = 0;
            for (;;) {
                bool have = true;
                uint64_t best = 0;
                for (int s = lane; s < cs; s += 64) {
                    const uint64_t v = ld_agent(&blk[s]);
                    if ((v & 15ull) != tag) have = false;
                    best = umax64(best, v);
                }
                if (__all(have)) { g = wave_max64(best) & ~15ull; break; }
                if ((++spins & 63u) == 0) {
                    if (aborted(y)) { ok = false; break; }
                    if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
                }
            }
        }
        if (lane == 0) { s_res = g; s_good = ok; }
    }
    __syncthreads();
    out = s_res;
    return s_good != 0;
}

// Whether every workgroup of the cluster runs on this workgroup's XCD, agreed
// by all of them through exchange number `e` (device-scope slots).  Before
// publishing its XCD id, each workgroup clears its own entries of the
// XCD-local slots `lslots` and waits until the clear has reached L2, so that
// once the answer is known no stale line of them can be read.  Returns 1 or
// 0, or -1 if the run was aborted; uniform over the workgroup.
__device__ int cluster_same_xcd(const Sync &y, uint64_t *slots, uint64_t *lslots, int slot_pad, int cs, int rank,
                                uint32_t e)
{
    __shared__ int s_same;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        const uint32_t me = xcc_id();
        const uint64_t tag = (uint64_t)((e & 7u) + 1u);
        uint64_t *blk = slots + (size_t)(e & 1u) * slot_pad;
        if (lane == 0) {
            st_xcd(&lslots[rank], 0);
            st_xcd(&lslots[slot_pad + rank], 0);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            st_agent(&blk[rank], ((uint64_t)me << 8) | tag);
        }
        int res = -1;
        const uint64_t t0 = wall_clock64();
        uint32_t spins = 0;
        for (;;) {
            bool have = true, same = true;
            for (int s = lane; s < cs; s += 64) {
                const uint64_t v = ld_agent(&blk[s]);
                if ((v & 15ull) != tag) have = false;
                else if ((uint32_t)((v >> 8) & 15ull) != me) same = false;
            }
            if (__all(have)) { res = __all(same) ? 1 : 0; break; }
            if ((++spins & 63u) == 0) {
                if (aborted(y)) break;
                if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); break; }
            }
        }
        if (lane == 0) s_same = res;
    }
    __syncthreads();
    return s_same;
}

// Two-level exchange for clusters spread over the XCDs (plain CLEAN's one
// cluster of cs >= 16 workgroups, rank r on XCD r % 8, checked at launch).
// Parity block: 8 XCD-local arrays of `hpad` slots, then 8 leader slots.
// Each workgroup publishes its key into its XCD's array with an XCD-local
// store; the XCD's leader (its lowest rank) takes their max and publishes it
// in its leader slot with a device-scope store; every workgroup polls the 8
// leader slots.  Two hops that stay short instead of one device-scope poll of
// every workgroup's slot, whose cost grows with the cluster.
__device__ bool cluster_reduce_xcd2(const Sync &y, uint64_t *hs, int hpad, int cs, int rank, uint32_t e,
                                    uint64_t tkey, uint64_t &out)
{
    __shared__ uint64_t s_wave[NWAVES];
    __shared__ uint64_t s_res;
    __shared__ int s_good;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t wk = wave_max64(tkey);
    if (lane == 0) s_wave[wave] = wk;
    __syncthreads();
    if (wave == 0) {
        uint64_t g = s_wave[0];
#pragma unroll
        for (int w = 1; w < NWAVES; ++w) g = umax64(g, s_wave[w]);
        bool ok = true;
        const uint64_t tag = (uint64_t)((e & 7u) + 1u);
        uint64_t *base = hs + (size_t)(e & 1u) * (8 * (size_t)hpad + 32);
        const int x = rank & 7, i = rank >> 3;
        uint64_t *lb = base + (size_t)x * hpad;
        uint64_t *gb = base + 8 * (size_t)hpad;
        if (lane == 0) st_xcd(&lb[i], (g & ~15ull) | tag);
        const uint64_t t0 = wall_clock64();
        uint32_t spins = 0;
        if (i == 0) {
            // the XCD's leader: its members' keys, then its leader slot
            const int nx = (cs - x + 7) >> 3;
            for (;;) {
                bool have = true;
                uint64_t best = 0;
                for (int s = lane; s < nx; s += 64) {
                    const uint64_t v = ld_agent(&lb[s]);
                    if ((v & 15ull) != tag) have = false;
                    best = umax64(best, v);
                }
                if (__all(have)) { g = wave_max64(best) & ~15ull; break; }
                if ((++spins & 63u) == 0) {
                    if (aborted(y)) { ok = false; break; }
                    if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
                }
            }
            if (ok && lane == 0) st_agent(&gb[x], g | tag);
        }
        // every workgroup: the leaders' keys
        const int nl = cs < 8 ? cs : 8;
        while (ok) {
            const uint64_t v = lane < nl ? ld_agent(&gb[lane]) : tag;
            if (__all((v & 15ull) == tag)) { g = wave_max64(lane < nl ? v : 0) & ~15ull; break; }
            if ((++spins & 63u) == 0) {
                if (aborted(y)) { ok = false; break; }
                if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
            }
        }
        if (lane == 0) { s_res = g; s_good = ok; }
    }
    __syncthreads();
    out = s_res;
    return s_good != 0;
}

// Whether rank r of a cluster runs on XCD r % 8 for every r (what the
// two-level exchange needs; plain launches place workgroup b on XCD b % 8),
// agreed through exchange `e` of the flat device-scope slots.  Before
// publishing, each workgroup clears its entries of the two-level XCD-local
// arrays (both parities) and waits until the clears have reached L2, so that
// no stale line of them can be read afterwards.  Returns 1 or 0, or -1 if the
// run was aborted; uniform over the workgroup.
__device__ int cluster_round_robin(const Sync &y, uint64_t *slots, int slot_pad, uint64_t *hs, int hpad, int cs,
                                   int rank, uint32_t e)
{
    __shared__ int s_rr;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave == 0) {
        const uint32_t me = xcc_id();
        const uint64_t tag = (uint64_t)((e & 7u) + 1u);
        uint64_t *blk = slots + (size_t)(e & 1u) * slot_pad;
        if (lane == 0) {
            const size_t at = (size_t)(rank & 7) * hpad + (size_t)(rank >> 3);
            st_xcd(&hs[at], 0);
            st_xcd(&hs[8 * (size_t)hpad + 32 + at], 0);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            st_agent(&blk[rank], ((uint64_t)(me == (uint32_t)(rank & 7)) << 8) | tag);
        }
        int res = -1;
        const uint64_t t0 = wall_clock64();
        uint32_t spins = 0;
        for (;;) {
            bool have = true, good = true;
            for (int s = lane; s < cs; s += 64) {
                const uint64_t v = ld_agent(&blk[s]);
                if ((v & 15ull) != tag) have = false;
                else if (!((v >> 8) & 1ull)) good = false;
            }
            if (__all(have)) { res = __all(good) ? 1 : 0; break; }
            if ((++spins & 63u) == 0) {
                if (aborted(y)) break;
                if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); break; }
            }
        }
        if (lane == 0) s_rr = res;
    }
    __syncthreads();
    return s_rr;
}

// Grid-wide barrier.  Data that crosses it is written and read with the
// agent-coherent accessors above; the barrier itself only orders: every wave
// waits for its own memory operations to complete, the workgroup barrier
// collects the waves, one agent-scope atomic arrives, and readers issue their
// loads only after they have seen all arrivals.
// `epoch` counts the barriers this workgroup has passed.  scope_barrier is
// the same over the `members` workgroups that share the counter `ctr` (one
// problem of a batch); grid_barrier is it over the whole grid.
__device__ bool scope_barrier(const Sync &y, uint32_t *ctr, uint32_t members, uint32_t &epoch, int *s_ok)
{
    // every wave's vector memory operations (its coherent stores) complete
    // before the workgroup can arrive
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    epoch += 1;
    if (threadIdx.x == 0) {
        bool ok = true;
        const uint32_t target = epoch * members;
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        while (ld_agent32(ctr) < target) {
            if (ld_agent32(&y.ctl->abort)) { ok = false; break; }
            if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
            __builtin_amdgcn_s_sleep(1);
        }
        *s_ok = ok;
    }
    __syncthreads();
    bool ok = *s_ok;
    __syncthreads();
    return ok;
}

__device__ __forceinline__ bool grid_barrier(const Sync &y, uint32_t &epoch, int *s_ok)
{
    return scope_barrier(y, &y.ctl->barrier, gridDim.x, epoch, s_ok);
}

// Two-level grid barrier for the rounds of a tiled launch.  One counter that
// every workgroup of the grid arrives on serialises the arrivals at the
// memory side (about 4 us for 256 workgroups, 9.5 us for 512); here a
// workgroup arrives on its XCD's counter, the last arriver of each XCD
// arrives on the leaders' counter, waits for every XCD that holds
// workgroups, and releases its XCD through a word of its own (about 2 us and
// 2.5 us).  The ordering argument is the flat barrier's: every wave's stores
// complete before its workgroup arrives, a leader arrives only after its whole
// XCD has, and a release is written only after every leader has arrived.
// x: this workgroup's XCD; mx: workgroups on it; nx: XCDs holding workgroups
// (both counted at launch); epoch counts these barriers.  The state lives in
// LDS and only thread 0 touches it, so it costs the persistent kernels no
// registers.
// FENCE adds an agent-scope release fence before the arrival and an acquire
// fence after the wait: plain (non-coherent) stores made before the barrier
// are then written back from the writer's L2, and plain loads after it miss
// every stale line in the reader's L1 and L2.  The transforms' column-major
// spectra use it: their 16-byte pieces of a line, written by the workgroups of
// one XCD, merge in that XCD's L2 instead of each going to memory on its own.
struct XcdBar {
    uint32_t x, mx, nx, epoch;
};

template <bool FENCE = false>
__device__ __forceinline__ bool xcd_grid_barrier(const Sync &y, XcdBar *xb, int *s_ok)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        if constexpr (FENCE) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool ok = true;
        const uint32_t x = xb->x, ep = xb->epoch + 1;
        xb->epoch = ep;
        uint32_t *rel = &y.ctl->xrel[x][0];
        const uint32_t old = __hip_atomic_fetch_add(&y.ctl->xarr[x][0], 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t t0 = wall_clock64();
        if (old + 1 == ep * xb->mx) {               // the last of this XCD
            __hip_atomic_fetch_add(&y.ctl->xlead, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t all = ep * xb->nx;
            while (ld_agent32(&y.ctl->xlead) < all) {
                if (ld_agent32(&y.ctl->abort)) { ok = false; break; }
                if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
                __builtin_amdgcn_s_sleep(1);
            }
            __hip_atomic_store(rel, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (ld_agent32(rel) < ep) {
                if (ld_agent32(&y.ctl->abort)) { ok = false; break; }
                if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); ok = false; break; }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if constexpr (FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_ok = ok;
    }
    __syncthreads();
    bool ok = *s_ok;
    __syncthreads();
    return ok;
}

__device__ __forceinline__ void tile_rect(const KArgs &a, int t, int &y0, int &x0, int &h, int &w)
{
    const int i = t / a.tx, j = t % a.tx;
    y0 = (int)((int64_t)i * a.ny / a.ty);
    const int y1 = (int)((int64_t)(i + 1) * a.ny / a.ty);
    x0 = (int)((int64_t)j * a.nx / a.tx);
    const int x1 = (int)((int64_t)(j + 1) * a.nx / a.tx);
    h = y1 - y0;
    w = x1 - x0;
}

// ------------------------------------------------- the register tile -----

// The arrays of one image.
struct Img {
    const float *dirty;
    float *residual;
    double *model;          // may be null
    float *accbuf;          // tiled feedback sums (image layout), else null
    float *rstart;          // FFT feedback: residual at the round's start, else null
    const void *psf;
    uint64_t psf_bytes;
    int nx, psf_nx, cy, cx;
};

// Residual held in VGPRs: thread t of cluster rank g owns K groups of V
// consecutive pixels, group k at tile-local index ((k*cs + g)*WG + t)*V.
template <int K, int V, typename PT> struct RegTile {
    static constexpr bool kResident = true;
    static constexpr bool kWide = false;
    static constexpr int kV = V;
    static constexpr int kPx = K * V;
    using psf_t = PT;
    float r[K][V];
    int32_t qoff[K];        // (y)*psf_nx + (x) of the group's first pixel, image coords
    uint64_t valid;         // bit k: group k inside the tile
    int y0, x0, h, w;       // tile rectangle
    int cs, rank;

    __device__ __forceinline__ uint32_t group_f(int k) const
    {
        return (uint32_t)(((k * cs + rank) * WG + (int)threadIdx.x) * V);
    }

    __device__ void init(const Img &a, int ty0, int tx0, int th, int tw, int ncs, int rk)
    {
        y0 = ty0; x0 = tx0; h = th; w = tw; cs = ncs; rank = rk;
        valid = 0;
        const int hw = h * w;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t f = group_f(k);
            if ((int64_t)f < hw) {
                valid |= 1ull << k;
                const int y = (int)(f / (uint32_t)w), x = (int)(f % (uint32_t)w);
                qoff[k] = (y0 + y) * a.psf_nx + (x0 + x);
                const int64_t img = (int64_t)(y0 + y) * a.nx + (x0 + x);
#pragma unroll
                for (int e = 0; e < V; ++e) r[k][e] = a.dirty[img + e];
                if (a.model) {
#pragma unroll
                    for (int e = 0; e < V; ++e) a.model[img + e] = 0.0;
                }
            } else {
                qoff[k] = 0;
#pragma unroll
                for (int e = 0; e < V; ++e) r[k][e] = 0.0f;
            }
        }
    }

    // Writes the residual out; returns this thread's sum of squares.
    __device__ double finish(const Img &a) const
    {
        double sumsq = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (valid & (1ull << k)) {
                const uint32_t f = group_f(k);
                const int y = (int)(f / (uint32_t)w), x = (int)(f % (uint32_t)w);
                const int64_t img = (int64_t)(y0 + y) * a.nx + (x0 + x);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    a.residual[img + e] = r[k][e];
                    sumsq += (double)r[k][e] * (double)r[k][e];
                }
            }
        }
        return sumsq;
    }

    // Thread-local peak key over the owned pixels: the largest |r|, then the
    // lowest index holding it.  Groups outside the tile hold +0 and come after
    // every valid group, so they never win unless all valid pixels are 0 too,
    // and then group 0 (valid) wins.  A NaN among the valid pixels outranks
    // everything: the lowest-index one is the key (a rare, terminal case,
    // detected by a NaN-propagating max beside the fast path).
    __device__ __forceinline__ uint64_t key(const Img &) const
    {
        if (!(valid & 1ull)) return 0;
        if constexpr (V == 4) {
            // one pass over the groups: the first group whose largest |r| is
            // the largest so far, with its four values, then the lowest of
            // those at that magnitude (a group holding a NaN has a NaN
            // maximum and is never taken here; no group taken: +0 at group 0)
            float gm = -1.0f;
            uint32_t kb = 0;
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float g = nan_max(nan_max(fabsf(r[k][0]), fabsf(r[k][1])), nan_max(fabsf(r[k][2]), fabsf(r[k][3])));
                // taken when larger, or NaN (unordered): a NaN group makes gm
                // NaN, which the slow path below handles
                const bool hit = !(g <= gm);
                gm = hit ? g : gm;
                kb = hit ? (uint32_t)k : kb;
                s0 = hit ? r[k][0] : s0;
                s1 = hit ? r[k][1] : s1;
                s2 = hit ? r[k][2] : s2;
                s3 = hit ? r[k][3] : s3;
            }
            if (__builtin_expect(is_nan(gm), 0)) return key_slow();
            uint32_t bb = __float_as_uint(s0), be = 0;
            if (gm >= 0.0f && fabsf(s0) != gm) {
                const bool h1 = fabsf(s1) == gm, h2 = fabsf(s2) == gm;
                bb = h1 ? __float_as_uint(s1) : h2 ? __float_as_uint(s2) : __float_as_uint(s3);
                be = h1 ? 1u : h2 ? 2u : 3u;
            }
            return make_key(bb, group_f((int)kb) + be);
        }
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) m = nan_max(m, fabsf(r[k][e]));
        if (__builtin_expect(is_nan(m), 0)) return key_slow();
        uint32_t bb = 0, bi = 0;
#pragma unroll
        for (int i = K * V - 1; i >= 0; --i) {
            const float x = r[i / V][i % V];
            const bool hit = fabsf(x) == m;
            bb = hit ? __float_as_uint(x) : bb;
            bi = hit ? (uint32_t)i : bi;
        }
        return make_key(bb, group_f((int)(bi / V)) + bi % V);
    }

    // The key when some group's maximum came out NaN.  A NaN among the valid
    // pixels makes the tile's peak non-finite: the key is a NaN (its position
    // is never used, as the run stops before appending).  Else the NaN sits in
    // a group outside the tile (which multiplies a PSF window by zero) and the
    // key is the largest |r| skipping NaN, as fmaxf does.  Rare and terminal.
    __device__ __forceinline__ uint64_t key_slow() const
    {
        bool vnan = false;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) vnan = vnan || (((valid >> k) & 1ull) && is_nan(r[k][e]));
        if (vnan) return make_key(0x7FC00000u, group_f(0));
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) m = fmaxf(m, fabsf(r[k][e]));
        uint32_t bb = 0, bi = 0;
#pragma unroll
        for (int i = K * V - 1; i >= 0; --i) {
            const float x = r[i / V][i % V];
            const bool hit = fabsf(x) == m;
            bb = hit ? __float_as_uint(x) : bb;
            bi = hit ? (uint32_t)i : bi;
        }
        return make_key(bb, group_f((int)(bi / V)) + bi % V);
    }

    // r -= c * PSF centred on image pixel (py, px); then, if asked, the new key.
    __device__ __forceinline__ uint64_t subtract(const Img &a, int py, int px, float c, bool want_key)
    {
        const int64_t w0 = (int64_t)(a.cy - py) * a.psf_nx + (a.cx - px);
        const char *base = (const char *)a.psf + w0 * (int64_t)sizeof(PT);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc_uniform(base, a.psf_bytes - (uint64_t)w0 * sizeof(PT));
        float pv[K][V];
#pragma unroll
        for (int k = 0; k < K; ++k) PsfLoad<PT, V>::load(rs, (uint32_t)qoff[k] * (uint32_t)sizeof(PT), pv[k]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float ck = (valid >> k) & 1ull ? c : 0.0f;    // groups outside the tile stay +0
#pragma unroll
            for (int e = 0; e < V; ++e) r[k][e] = __builtin_fmaf(-ck, pv[k][e], r[k][e]);
        }
        return want_key ? key(a) : 0;
    }

    // r -= acc (float32 feedback sums, image layout); FROM_START (FFT form,
    // acc holds every tile's contribution): r = rstart - acc, and rstart = r.
    // Returns the new key.  Only the owning thread touches rstart.
    template <bool FROM_START> __device__ __forceinline__ uint64_t apply_feedback(const Img &a)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (valid & (1ull << k)) {
                const uint32_t f = group_f(k);
                const int y = (int)(f / (uint32_t)w), x = (int)(f % (uint32_t)w);
                const int64_t img = (int64_t)(y0 + y) * a.nx + (x0 + x);
                if constexpr (FROM_START) {
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        r[k][e] = a.rstart[img + e] - ldc(&a.accbuf[img + e]);
                        a.rstart[img + e] = r[k][e];
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e) r[k][e] = r[k][e] - ldc(&a.accbuf[img + e]);
                }
            }
        }
        return key(a);
    }

    // Does this thread own tile-local index f?
    __device__ __forceinline__ bool owns(uint32_t f) const
    {
        const uint32_t u = f / (uint32_t)V;
        const uint32_t t = u % (uint32_t)WG;
        const uint32_t g = (u / (uint32_t)WG) % (uint32_t)cs;
        return t == threadIdx.x && (int)g == rank;
    }
};

// Running peak of a stream of pixels in increasing index order: the largest
// |value| (compared as magnitude bits, every NaN one value above +Inf), the
// lowest index on ties.
__device__ __forceinline__ void take_key(uint32_t bits, uint32_t f, uint32_t &bb, uint32_t &bf, bool &any)
{
    const bool t = !any || peak_mag(bits) > peak_mag(bb);
    bb = t ? bits : bb;
    bf = t ? f : bf;
    any = true;
}

// Residual held in VGPRs at 128 pixels per thread during each round's local
// loops, for images too large for RegTile's shapes: one 512-thread workgroup
// per CU holds 64K pixels, so the co-resident grid holds 16M (a 4096^2
// image).  Thread t of cluster rank g owns 32 groups of 4 pixels at
// tile-local index f_k = f_0 + k*S, with f_0 = (g*WG + t)*4 and S = cs*WG*4
// a multiple of the tile width w: group k sits k*S/w rows below group 0, so
// one PSF offset plus a uniform step addresses all 32.  Groups
// 0..nvalid-1 lie inside the tile; the others hold +0.
//
// Only wide_round() holds the residual in registers, loading it at the
// start of each round's local loops from the round's residual array (the FFT
// form's rstart, else `residual`) and, for the direct gather, storing it back
// at their end.  Everything else (the first peak, applying the feedback, the
// final write) streams those arrays like StreamTile, so the feedback phases
// never carry 128 residual registers.
template <typename PT> struct WideTile {
    static constexpr bool kResident = false;
    static constexpr bool kWide = true;
    static constexpr int kV = 4;
    static constexpr int K = 32, V = 4;
    using psf_t = PT;
    int32_t qoff;           // PSF offset (image coords) of group 0's first pixel
    int32_t f0;             // tile-local index of group 0's first pixel
    int nvalid;             // groups inside the tile
    int y0, x0, h, w, cs, rank;
    bool fft;               // the round's residual lives in rstart (else residual)

    __device__ __forceinline__ uint32_t stride() const { return (uint32_t)(cs * WG * V); }
    __device__ __forceinline__ uint32_t group_f(int k) const { return (uint32_t)f0 + (uint32_t)k * stride(); }
    __device__ __forceinline__ int64_t img_of(const Img &a, int k) const
    {
        const int y = f0 / w + k * (int)(stride() / (uint32_t)w), x = f0 % w;
        return (int64_t)(y0 + y) * a.nx + (x0 + x);
    }
    __device__ __forceinline__ float *cur(const Img &a) const { return fft ? a.rstart : a.residual; }

    // Geometry; the direct gather's residual array starts as the dirty image
    // (data: also that first copy and the model's zeros, once per tile).
    __device__ void init(const Img &a, int ty0, int tx0, int th, int tw, int ncs, int rk, bool data = true)
    {
        y0 = ty0; x0 = tx0; h = th; w = tw; cs = ncs; rank = rk;
        fft = a.rstart != nullptr;
        f0 = (rank * WG + (int)threadIdx.x) * V;
        const int hw = h * w;
        nvalid = f0 < hw ? min(K, (int)(((uint32_t)(hw - f0) + stride() - 1) / stride())) : 0;
        qoff = (y0 + f0 / w) * a.psf_nx + (x0 + f0 % w);
        if (!data) return;
        for (int k = 0; k < nvalid; ++k) {
            const int64_t img = img_of(a, k);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if (!fft) a.residual[img + e] = a.dirty[img + e];
                if (a.model) a.model[img + e] = 0.0;
            }
        }
    }

    // Thread-local peak key of the round's residual array, streamed.
    __device__ uint64_t key(const Img &a) const
    {
        const float *rr = cur(a);
        uint32_t bb = 0, bf = 0;
        bool any = false;
        for (int k = 0; k < nvalid; ++k) {
            const int64_t img = img_of(a, k);
#pragma unroll
            for (int e = 0; e < V; ++e) take_key(__float_as_uint(rr[img + e]), group_f(k) + e, bb, bf, any);
        }
        return any ? make_key(bb, bf) : 0;
    }

    // r = array - acc for every owned pixel, written back; returns the new key.
    template <bool FROM_START> __device__ uint64_t apply_feedback(const Img &a)
    {
        float *rr = cur(a);
        uint32_t bb = 0, bf = 0;
        bool any = false;
        for (int k = 0; k < nvalid; ++k) {
            const int64_t img = img_of(a, k);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const float r = rr[img + e] - ldc(&a.accbuf[img + e]);
                rr[img + e] = r;
                take_key(__float_as_uint(r), group_f(k) + e, bb, bf, any);
            }
        }
        return any ? make_key(bb, bf) : 0;
    }

    __device__ double finish(const Img &a) const
    {
        const float *rr = cur(a);
        double sumsq = 0.0;
        for (int k = 0; k < nvalid; ++k) {
            const int64_t img = img_of(a, k);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const float r = rr[img + e];
                if (fft) a.residual[img + e] = r;
                sumsq += (double)r * (double)r;
            }
        }
        return sumsq;
    }

    __device__ __forceinline__ bool owns(uint32_t f) const
    {
        const uint32_t u = (f % stride()) / (uint32_t)V;
        return u % (uint32_t)WG == threadIdx.x && (int)(u / (uint32_t)WG) == rank;
    }
};

// What one round's local loops of a WideTile cluster leave behind.
struct WideRound {
    uint64_t cur;           // the cluster's last peak key
    uint32_t e;             // exchanges so far
    int L;                  // components found
    int ok;                 // 0: the run was aborted
};

// One round's local loops of a WideTile cluster (the same steps as the
// register tiles' loop in tiled_kernel), in a function of its own so that its
// 128 residual registers do not add to the rest of the kernel's.  The
// residual comes from the round's residual array and, for the direct gather,
// goes back to it at the end (the FFT form rebuilds it from the round's start).
// FULL: the tile fills every group of every thread (its pixels are exactly
// cs * WG * 4 * 32), so no group needs a test of whether it lies inside the
// tile.  Such tests are loop-invariant per group, and the compiler hoists
// them out of the minor loop into 32 mask registers that no longer fit.
template <typename PT, bool FULL>
__device__ __noinline__ WideRound wide_round(const KArgs &a, const Img im, const WideTile<PT> R, const Sync y,
                                             uint64_t *slots, uint64_t *lslots, uint32_t e, uint64_t cur,
                                             int64_t budget, double level, bool leader, int32_t *l_idx,
                                             float *l_flux)
{
    constexpr int K = WideTile<PT>::K, V = WideTile<PT>::V;
    float r[K][V];
    const float *src = R.cur(im);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int64_t img = R.img_of(im, k);
#pragma unroll
        for (int e2 = 0; e2 < V; ++e2) r[k][e2] = (FULL || k < R.nvalid) ? src[img + e2] : 0.0f;
    }
    // the round's scalars (equal in every lane) in scalar registers: this
    // function's arguments and what is read through them are vector values
    // to the compiler
    const double thr = wave_uniform(a.threshold), lvl = wave_uniform(level);
    const float gain = wave_uniform(a.gain);
    const int anx = wave_uniform(a.nx), acy = wave_uniform(a.cy), acx = wave_uniform(a.cx);
    const int apnx = wave_uniform(a.psf_nx), tw = wave_uniform(R.w), ty0 = wave_uniform(R.y0), tx0 = wave_uniform(R.x0);
    const void *psf = wave_uniform(a.psf);
    const void *psf1 = wave_uniform(a.psf1);
    const uint64_t psf_bytes = wave_uniform(a.psf_bytes);
    double *model = wave_uniform(a.model);
    const int64_t nb = wave_uniform(budget);
    const uint32_t voff = (uint32_t)R.qoff * (uint32_t)sizeof(PT);
    const uint32_t step = wave_uniform((R.stride() / (uint32_t)tw) * (uint32_t)apnx * (uint32_t)sizeof(PT));
    WideRound out{wave_uniform(cur), e, 0, 1};
    for (int64_t it = 0; it < nb; ++it) {
        const float v = key_value(out.cur);
        if (!__builtin_isfinite(v) || (double)fabsf(v) < thr || (double)fabsf(v) < lvl) break;
        const float c = gain * v;
        const uint32_t fp = key_f(out.cur);
        // the division runs on the vector unit; its result goes back to
        // scalar registers, so that the 32 descriptors below are scalar work
        const int ly = wave_uniform((int)(fp / (uint32_t)tw)), lx = wave_uniform((int)(fp % (uint32_t)tw));
        const int py = ty0 + ly, px = tx0 + lx;
        const int32_t img = py * anx + px;
        if (leader && threadIdx.x == 0) { l_idx[out.L] = img; l_flux[out.L] = c; }
        if (model && R.owns(fp)) model[img] += (double)c;
        // r -= c * PSF window (eq. 2).  The loads go out WB at a time, on
        // one descriptor per batch (base: the batch's first group's window,
        // in scalar registers) with group k0 + j at scalar offset j * step and
        // the thread's own offset in the vector offset.  Groups outside the
        // tile take a vector offset past any range, so their loads read 0 and
        // touch no memory; they are multiplied by 0.  (With the 32 group
        // offsets held in vector registers instead, the compiler had waited
        // for each load before issuing the next.)
        uint64_t wb = (uint64_t)((int64_t)(acy - py) * apnx + (acx - px)) * sizeof(PT);
        // an FP16 window at an odd element is read from the copy moved down
        // one element, where it starts on a 4-byte boundary (8-byte loads at
        // 2-byte-aligned addresses cost the memory pipeline about what the
        // FP32 window's 16 bytes do)
        const char *pbase = (const char *)psf;
        if (sizeof(PT) == 2 && psf1 != nullptr && (wb & 2) != 0) {
            pbase = (const char *)psf1;
            wb -= 2;
        }
        constexpr int WB = 16;
        constexpr uint32_t kOutside = 0xFFFFFFF0u;
        // the group offsets j * step are made here, in each iteration, from
        // a step the compiler cannot see through: hoisted out of the loop,
        // 15 of them would hold scalar registers the loop runs short of
        uint32_t st = step;
        asm volatile("" : "+s"(st));
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += WB) {
            const uint64_t kb = wb + (uint64_t)k0 * st;
            // the range stops short of kOutside, whatever the PSF's size
            const uint32_t nrec = min(clamp_u32((int64_t)(psf_bytes - kb)), kOutside - 1u);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void *)(pbase + kb), (short)0, (int)nrec, 0x00020000);
            float pv[WB][V];
#pragma unroll
            for (int j = 0; j < WB; ++j)
                PsfLoad<PT, V>::load_s(rs, (FULL || k0 + j < R.nvalid) ? voff : kOutside, (uint32_t)j * st, pv[j]);
#pragma unroll
            for (int j = 0; j < WB; ++j) {
                const float ck = (FULL || k0 + j < R.nvalid) ? c : 0.0f;      // groups outside the tile stay +0
#pragma unroll
                for (int e2 = 0; e2 < V; ++e2) r[k0 + j][e2] = __builtin_fmaf(-ck, pv[j][e2], r[k0 + j][e2]);
            }
        }
        out.L += 1;
        if (it + 1 < nb) {
            // thread key: the largest |r|, then the lowest index holding it
            // (the same as take_key's).  One pass over the groups keeps the
            // first group whose largest |r| is the largest so far, with its
            // four values; then the lowest of those four at that magnitude.
            // A group holding a NaN has a NaN maximum and is never taken
            // there; a NaN-propagating max beside it sends that rare,
            // terminal case to a scan for the lowest-index NaN.
            float m = -1.0f;
            uint32_t kb = 0;
            float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float g = nan_max(nan_max(fabsf(r[k][0]), fabsf(r[k][1])), nan_max(fabsf(r[k][2]), fabsf(r[k][3])));
                const bool hit = !(g <= m);             // larger, or NaN
                m = hit ? g : m;
                kb = hit ? (uint32_t)k : kb;
                s0 = hit ? r[k][0] : s0;
                s1 = hit ? r[k][1] : s1;
                s2 = hit ? r[k][2] : s2;
                s3 = hit ? r[k][3] : s3;
            }
            uint32_t bb = __float_as_uint(s0), be = 0;      // no group taken: (+0, group 0)
            if (m >= 0.0f && fabsf(s0) != m) {
                const bool h1 = fabsf(s1) == m, h2 = fabsf(s2) == m;
                bb = h1 ? __float_as_uint(s1) : h2 ? __float_as_uint(s2) : __float_as_uint(s3);
                be = h1 ? 1u : h2 ? 2u : 3u;
            }
            uint64_t tk = R.nvalid > 0 ? make_key(bb, R.group_f((int)kb) + be) : 0;
            if (__builtin_expect(is_nan(m), 0)) {
                // a group's maximum is NaN: a NaN in a group inside the tile
                // makes the peak non-finite (the key is a NaN; its position is
                // never used); else the NaN is in a group past the tile's end
                // (which multiplies a PSF window by zero) and the key is the
                // largest |r| skipping NaN
                bool vnan = false;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    vnan = vnan || ((FULL || k < R.nvalid) && is_nan(nan_max(nan_max(r[k][0], r[k][1]), nan_max(r[k][2], r[k][3]))));
                if (vnan) {
                    tk = make_key(0x7FC00000u, R.group_f(0));
                } else {
                    float m2 = -1.0f;
                    uint32_t k2 = 0;
                    float t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const float g = fmaxf(fmaxf(fabsf(r[k][0]), fabsf(r[k][1])), fmaxf(fabsf(r[k][2]), fabsf(r[k][3])));
                        const bool hit = g > m2;
                        m2 = hit ? g : m2;
                        k2 = hit ? (uint32_t)k : k2;
                        t0 = hit ? r[k][0] : t0;
                        t1 = hit ? r[k][1] : t1;
                        t2 = hit ? r[k][2] : t2;
                        t3 = hit ? r[k][3] : t3;
                    }
                    uint32_t b2 = __float_as_uint(t0), e2 = 0;
                    if (m2 >= 0.0f && fabsf(t0) != m2) {
                        const bool h1 = fabsf(t1) == m2, h2 = fabsf(t2) == m2;
                        b2 = h1 ? __float_as_uint(t1) : h2 ? __float_as_uint(t2) : __float_as_uint(t3);
                        e2 = h1 ? 1u : h2 ? 2u : 3u;
                    }
                    tk = R.nvalid > 0 ? make_key(b2, R.group_f((int)k2) + e2) : 0;
                }
            }
            if (!cluster_reduce(y, slots, lslots, a.slot_pad, R.cs, R.rank, out.e++, tk, out.cur)) {
                out.ok = 0;
                return out;
            }
            out.cur = wave_uniform(out.cur);
        }
    }
    if (!R.fft) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (FULL || k < R.nvalid) {
                const int64_t img = R.img_of(im, k);
#pragma unroll
                for (int e2 = 0; e2 < V; ++e2) im.residual[img + e2] = r[k][e2];
            }
        }
    }
    return out;
}

// Residual kept in HBM (the caller's residual array) for tiles too large for
// the register file: every pass streams K groups per thread through
// registers, group index ((p*K + k)*cs + g)*WG + t for pass p.
template <int K, int V, typename PT> struct StreamTile {
    static constexpr bool kResident = false;
    static constexpr bool kWide = false;
    static constexpr int kV = V;
    using psf_t = PT;
    int y0, x0, h, w, cs, rank, passes;

    __device__ __forceinline__ uint32_t group_f(int p, int k) const
    {
        return (uint32_t)((((p * K + k) * cs + rank) * WG + (int)threadIdx.x) * V);
    }
    __device__ __forceinline__ int64_t img_of(const Img &a, uint32_t f) const
    {
        const int y = (int)(f / (uint32_t)w), x = (int)(f % (uint32_t)w);
        return (int64_t)(y0 + y) * a.nx + (x0 + x);
    }

    __device__ void init(const Img &a, int ty0, int tx0, int th, int tw, int ncs, int rk)
    {
        y0 = ty0; x0 = tx0; h = th; w = tw; cs = ncs; rank = rk;
        const int64_t per_pass = (int64_t)K * cs * WG * V;
        passes = (int)(((int64_t)h * w + per_pass - 1) / per_pass);
        const int64_t hw = (int64_t)h * w;
        for (int p = 0; p < passes; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = group_f(p, k);
                if ((int64_t)f >= hw) continue;
                const int64_t img = img_of(a, f);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    if (a.residual != a.dirty) a.residual[img + e] = a.dirty[img + e];
                    if (a.model) a.model[img + e] = 0.0;
                }
            }
    }

    __device__ double finish(const Img &a) const
    {
        double sumsq = 0.0;
        const int64_t hw = (int64_t)h * w;
        for (int p = 0; p < passes; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = group_f(p, k);
                if ((int64_t)f >= hw) continue;
                const int64_t img = img_of(a, f);
#pragma unroll
                for (int e = 0; e < V; ++e) sumsq += (double)a.residual[img + e] * (double)a.residual[img + e];
            }
        return sumsq;
    }

    __device__ __forceinline__ static void take(uint32_t bits, uint32_t f, uint32_t &bb, uint32_t &bf, bool &any)
    {
        const bool t = !any || peak_mag(bits) > peak_mag(bb);
        bb = t ? bits : bb;
        bf = t ? f : bf;
        any = true;
    }

    __device__ uint64_t key(const Img &a) const
    {
        uint32_t bb = 0, bf = 0;
        bool any = false;
        const int64_t hw = (int64_t)h * w;
        for (int p = 0; p < passes; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = group_f(p, k);
                if ((int64_t)f >= hw) continue;
                const int64_t img = img_of(a, f);
#pragma unroll
                for (int e = 0; e < V; ++e) take(__float_as_uint(a.residual[img + e]), f + e, bb, bf, any);
            }
        return any ? make_key(bb, bf) : 0;
    }

    __device__ uint64_t subtract(const Img &a, int py, int px, float c, bool want_key)
    {
        const int64_t w0 = (int64_t)(a.cy - py) * a.psf_nx + (a.cx - px);
        const char *base = (const char *)a.psf + w0 * (int64_t)sizeof(PT);
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, a.psf_bytes - (uint64_t)w0 * sizeof(PT));
        uint32_t bb = 0, bf = 0;
        bool any = false;
        const int64_t hw = (int64_t)h * w;
        for (int p = 0; p < passes; ++p) {
            float rv[K][V], pv[K][V];
            int64_t img[K];
            bool ok[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = group_f(p, k);
                ok[k] = (int64_t)f < hw;
                const int y = (int)(f / (uint32_t)w), x = (int)(f % (uint32_t)w);
                img[k] = (int64_t)(y0 + y) * a.nx + (x0 + x);
                const uint32_t qo = (uint32_t)((y0 + y) * a.psf_nx + (x0 + x));
                if (ok[k]) {
                    PsfLoad<PT, V>::load(rs, qo * (uint32_t)sizeof(PT), pv[k]);
#pragma unroll
                    for (int e = 0; e < V; ++e) rv[k][e] = a.residual[img[k] + e];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (!ok[k]) continue;
                const uint32_t f = group_f(p, k);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const float r = __builtin_fmaf(-c, pv[k][e], rv[k][e]);
                    a.residual[img[k] + e] = r;
                    if (want_key) take(__float_as_uint(r), f + e, bb, bf, any);
                }
            }
        }
        return any ? make_key(bb, bf) : 0;
    }

    template <bool FROM_START> __device__ uint64_t apply_feedback(const Img &a)
    {
        uint32_t bb = 0, bf = 0;
        bool any = false;
        const int64_t hw = (int64_t)h * w;
        for (int p = 0; p < passes; ++p)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = group_f(p, k);
                if ((int64_t)f >= hw) continue;
                const int64_t img = img_of(a, f);
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const float r = (FROM_START ? a.rstart[img + e] : a.residual[img + e]) - ldc(&a.accbuf[img + e]);
                    a.residual[img + e] = r;
                    if constexpr (FROM_START) a.rstart[img + e] = r;
                    take(__float_as_uint(r), f + e, bb, bf, any);
                }
            }
        return any ? make_key(bb, bf) : 0;
    }

    __device__ __forceinline__ bool owns(uint32_t f) const
    {
        const uint32_t u = f / (uint32_t)V;
        const uint32_t t = u % (uint32_t)WG;
        const uint32_t g = (u / (uint32_t)WG) % (uint32_t)cs;
        return t == threadIdx.x && (int)g == rank;
    }
};

// ------------------------------------------------------ plain kernel -----

// Sum of the workgroup's squared residuals, in a fixed order, to partial[slot].
template <class Tile> __device__ void store_and_sum(const Tile &R, const Img &im, double *partial, int slot)
{
    __shared__ double s_ss[NWAVES];
    double ss = R.finish(im);
    ss = wave_sum64f(ss);
    if ((threadIdx.x & 63) == 0) s_ss[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < NWAVES; ++w) tot += s_ss[w];
        partial[slot] = tot;
    }
    __syncthreads();
}

// Plain Hogbom CLEAN of one image by a cluster of j.cs workgroups; this
// workgroup is cluster rank `rank`.  `local`: the whole cluster runs on this
// XCD, so after the first exchange keys go through the XCD-local slots (each
// member clears its entries of them before that first, device-scope
// exchange, which no member passes until all have cleared theirs).  Returns
// false if the run was aborted.
// `cancel`: the caller's flag (host memory) or null; `hslots`/`hpad`: the
// two-level exchange slots of a large plain cluster, or null.
template <class Tile>
__device__ __forceinline__ bool run_plain(const PlainJob &j_arg, int rank_arg, const Sync &y, bool local,
                                          const int32_t *cancel, uint64_t *hslots, int hpad)
{
    const PlainJob j = wave_uniform(j_arg);     // one problem per workgroup
    const int rank = wave_uniform(rank_arg);
    const Img im{j.dirty, j.residual, j.model, nullptr, nullptr, j.psf, j.psf_bytes, j.nx, j.psf_nx, j.cy, j.cx};
    Tile T;
    T.init(im, 0, 0, j.ny, j.nx, j.cs, rank);
    if (!Tile::kResident) __syncthreads();

    uint64_t *ls = nullptr;
    if (local) {
        if (threadIdx.x == 0) {
            st_xcd(&j.lslots[rank], 0);
            st_xcd(&j.lslots[j.slot_pad + rank], 0);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        ls = j.lslots;
    }
    uint32_t e = 0;
    // a large cluster spread over the XCDs (plain CLEAN) exchanges in two
    // levels when every rank sits on the XCD the placement intends
    bool two = false;
    if (hslots) {
        const int rr = cluster_round_robin(y, j.slots, j.slot_pad, hslots, hpad, j.cs, rank, e++);
        if (rr < 0) return false;
        two = rr > 0;
    }
    uint64_t cur;
    if (!cluster_reduce(y, j.slots, nullptr, j.slot_pad, j.cs, rank, e++, T.key(im), cur)) return false;
    cur = wave_uniform(cur);

    const bool leader = rank == 0 && threadIdx.x == 0;
    int64_t n = 0;
    int32_t stop;
    double mflux = 0.0;
    for (;;) {
        // peak (eq. 1): value and position from the cluster's key
        const float v = key_value(cur);
        if (n == j.max_iter) { stop = STOP_MAXITER; break; }
        if (cancel && n % CANCEL_EVERY == 0) {
            // cancel checkpoint: rank 0 reads the caller's flag and the
            // cluster takes the max, so every member stops at the same n
            const uint64_t vote = rank == 0 && threadIdx.x == 0 && host_flag(cancel) ? (1ull << 33) : 0ull;
            uint64_t got;
            if (!(two ? cluster_reduce_xcd2(y, hslots, hpad, j.cs, rank, e++, vote, got)
                      : cluster_reduce(y, j.slots, ls, j.slot_pad, j.cs, rank, e++, vote, got)))
                return false;
            if (got) { stop = STOP_CANCELLED; break; }
        }
        if (!__builtin_isfinite(v)) { stop = STOP_NONFINITE; break; }
        if ((double)fabsf(v) < j.threshold) { stop = STOP_THRESHOLD; break; }
        if (n == j.cap) { stop = STOP_CAPACITY; break; }
        const float c = j.gain * v;
        const uint32_t fp = key_f(cur);
        const int py = (int)(fp / (uint32_t)j.nx), px = (int)(fp % (uint32_t)j.nx);
        if (leader) {
            j.comp_idx[n] = (int32_t)fp;
            j.comp_flux[n] = c;
            mflux += (double)c;
        }
        if (j.model && T.owns(fp)) j.model[fp] += (double)c;
        // subtraction (eq. 2) fused with the next peak search
        const uint64_t tk = T.subtract(im, py, px, c, true);
        if (!(two ? cluster_reduce_xcd2(y, hslots, hpad, j.cs, rank, e++, tk, cur)
                  : cluster_reduce(y, j.slots, ls, j.slot_pad, j.cs, rank, e++, tk, cur)))
            return false;
        cur = wave_uniform(cur);
        n += 1;
    }
    store_and_sum(T, im, j.partial, rank);
    if (leader) {
        j.dstat->n_iter = n;
        j.dstat->stop = stop;
        j.dstat->n_rounds = 0;
        j.dstat->final_peak = (double)key_value(cur);
        j.dstat->model_flux = mflux;
        j.dstat->xcd_local = local ? 1 : 0;
        j.dstat->levels = two ? 2 : 1;
    }
    return true;
}

template <class Tile> __global__ void __launch_bounds__(WG) hogbom_kernel(const KArgs a)
{
    const int32_t role = a.role[blockIdx.x];
    if (role < 0) return;                       // no helpers in the plain form
    const Sync y{a.ctl, a.timeout_ticks};
    PlainJob j;
    j.dirty = a.dirty; j.residual = a.residual; j.model = a.model;
    j.psf = a.psf; j.psf_bytes = a.psf_bytes;
    j.ny = a.ny; j.nx = a.nx; j.psf_nx = a.psf_nx; j.cy = a.cy; j.cx = a.cx;
    j.gain = a.gain; j.threshold = a.threshold; j.max_iter = a.max_iter; j.cap = a.cap;
    j.comp_idx = a.comp_idx; j.comp_flux = a.comp_flux;
    j.slots = a.xslots; j.lslots = nullptr; j.slot_pad = a.slot_pad; j.cs = a.cs;
    j.dstat = a.dstat; j.partial = a.partial;
    run_plain<Tile>(j, role & 0xFFFF, y, false, a.cancel, a.hslots, a.hpad);
}

// Ticket of the per-XCD schedule: the problem and cluster rank this
// workgroup (on XCD x) takes next, or -1 when none is left.  Tickets of one
// XCD go out in order; the holder of the first unassigned ticket (the front)
// pulls the next problem of the batch, writes its cs tickets and moves the
// front on.  Thread 0 only.
__device__ int32_t xcd_ticket(const BatchArgs &b, const Sync &y, uint32_t x)
{
    XcdQueue *q = b.xq;
    int32_t *table = b.xtable + (size_t)x * b.tickets;
    const uint32_t t = __hip_atomic_fetch_add(&q->next[x * XQ_STRIDE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    uint32_t spins = 0;
    for (;;) {
        uint32_t f = ld_agent32(&q->front[x * XQ_STRIDE]);
        if (t < f) return ldc(&table[t]);
        if (t == f) {
            const uint32_t p = __hip_atomic_fetch_add(&q->problem[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int)p >= b.n) {
                stc(&q->closed[x * XQ_STRIDE], 1u);
                return -1;
            }
            const int cs = b.jobs[p].cs;
            for (int r = 0; r < cs; ++r) stc(&table[t + r], (int32_t)((p << 12) | (uint32_t)r));
            // the table entries land before the front that publishes them
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            stc(&q->front[x * XQ_STRIDE], t + (uint32_t)cs);
            return (int32_t)(p << 12);
        }
        // t > f: wait for the front, or for the queue to close (re-reading
        // the front: it may have passed t before the close)
        if (ld_agent32(&q->closed[x * XQ_STRIDE])) {
            f = ld_agent32(&q->front[x * XQ_STRIDE]);
            return t < f ? ldc(&table[t]) : -1;
        }
        if ((++spins & 63u) == 0) {
            if (aborted(y)) return -1;
            if (wall_clock64() - t0 > y.timeout_ticks) { raise_abort(y, ABORT_TIMEOUT); return -1; }
        }
    }
}

// ----------------------------------------------------- FFT feedback -----
//
// The feedback step in FFT form: per round, the residual becomes the round's
// starting residual minus (the round's component image (*) the PSF), one
// circular convolution on an Ly x Lx grid (powers of two >= 2n - 1, so the
// image window sees no wrap-around).  The component image is real: rows go
// two at a time through one complex transform along x, and only the
// Lx/2 + 1 non-redundant bins are carried through the y transforms.
//
// An axis of length L <= 8192 is transformed in one pass in LDS (one
// transform per workgroup).  Longer axes use two levels, L = L1 * L2 with
// n = L2 n1 + n2 and k = k1 + L1 k2 (the four-step scheme): transforms of
// length L1 over n1 (strided), times W_L^(n2 k1), then transforms of length
// L2 over n2 (contiguous); the inverse runs the same steps backwards.  The
// two-level spectra come out in (k1, k2) order; the PSF kernel's spectrum is
// computed once per call by the same code, so both orders agree.

// Loads in flight per thread in the two-level phases: enough to overlap their
// round trips, few enough to keep the streamed FFT kernel within 128 VGPRs.
constexpr int STAGE_TWO = 4;
// The same in the wide-tile kernel, whose transform phases run at one
// workgroup per CU in functions with the whole register file to themselves:
// half the waves to hide the round trips, and the registers for more.
constexpr int STAGE_TWO_WIDE = 16;

struct FftAxis {
    int lg, L, H;           // length 2^lg; H = L/2 + 1 (x axis: carried bins)
    bool two;               // two levels: L = L1 * L2
    int lg1, lg2, L1, L2;
    const float2 *tw;       // W_L^m, m < L
};

__device__ __forceinline__ FftAxis fft_axis(int lg, int two, const float2 *tw)
{
    FftAxis f;
    f.lg = lg;
    f.L = 1 << lg;
    f.H = f.L / 2 + 1;
    f.two = two != 0;
    f.tw = tw;
    f.lg1 = lg / 2;
    f.lg2 = lg - f.lg1;
    f.L1 = 1 << f.lg1;
    f.L2 = 1 << f.lg2;
    return f;
}

// log2 of the number of strided length-L1 transforms one workgroup holds in
// LDS at a time (segments padded to L1 + 1 against bank conflicts).
__device__ __forceinline__ int strided_block_lg(const FftAxis &f)
{
    int lg = 0;
    while (lg < f.lg2 && (2 << lg) * fft_seg_stride(f.L1) <= FFT_LDS_CPLX) ++lg;
    return lg;
}

// Carried column of x bin (k1, k2), two levels: bins k = k1 + L1 k2 <= L/2,
// laid out k1-major (L2/2 per row k1) with k = L/2 last.
__device__ __forceinline__ int chat_of(const FftAxis &f, int k1, int k2)
{
    return k2 < f.L2 / 2 ? k1 * (f.L2 / 2) + k2 : f.L / 2;
}

// The bin holding index L - k (two levels).
__device__ __forceinline__ void mirror_of(const FftAxis &f, int k1, int k2, int &q1, int &q2)
{
    if (k1 == 0) {
        q1 = 0;
        q2 = (f.L2 - k2) & (f.L2 - 1);
    } else {
        q1 = f.L1 - k1;
        q2 = f.L2 - 1 - k2;
    }
}

// Value of the PSF kernel image at grid point (row, x): K(d) = psf[centre + d]
// for |d| < (ny, nx), placed circularly, zero elsewhere.
template <typename PT>
__device__ __forceinline__ float kernel_value(const KArgs &a, int Ly, int Lx, int row, int x)
{
    const int dy = row < a.ny ? row : row - Ly;
    const int dx = x < a.nx ? x : x - Lx;
    if (dy <= -a.ny || dx <= -a.nx) return 0.0f;
    return (float)((const PT *)a.psf)[(int64_t)(a.cy + dy) * a.psf_nx + (a.cx + dx)];
}

// Tile row / column of an image row / column (floor split).
__device__ __forceinline__ int tile_row_of(const KArgs &a, int y)
{
    int i = (int)((int64_t)y * a.ty / a.ny);
    while (i + 1 < a.ty && (int)((int64_t)(i + 1) * a.ny / a.ty) <= y) ++i;
    while (i > 0 && (int)((int64_t)i * a.ny / a.ty) > y) --i;
    return i;
}

// Split of a row pair's transform Z (row r0 real part, r0+1 imaginary part)
// at bin k: A = (Z[k] + conj Z[L-k]) / 2 and B = (Z[k] - conj Z[L-k]) / 2i,
// stored column-major for the y phase: bin k of rows r0 and r0 + 1 at
// o[k * rows] and o[k * rows + 1] (o = buffer + r0), plain stores (a fenced
// barrier follows); one 16-byte store when `rows` is even (row r0 + 1 then
// always exists and the pair is 16-byte aligned).
__device__ __forceinline__ void store_cols(float2 *o, int rows, bool has1, int k, float2 zk, float2 zm)
{
    const float2 v0 = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 v1 = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    float2 *p = o + (size_t)k * rows;
    if ((rows & 1) == 0) {
        stp4(p, v0, v1);
    } else {
        stp2(p, v0);
        if (has1) stp2(p + 1, v1);
    }
}

// The x phases' row-pair order: the workgroups of one XCD
// (workgroup b runs on XCD b % 8) take consecutive row pairs, so that the
// 16-byte pieces of one column-major line are written, and read, through a
// single L2.  Any order is correct; this is the one-to-one map of
// [0, gridDim.x) that groups them (the identity when the grid is not a
// multiple of 8).
__device__ __forceinline__ int xcd_slot()
{
    const int w = blockIdx.x, g = gridDim.x;
    return (g & 7) ? w : (w & 7) * (g >> 3) + (w >> 3);
}

// x forward, one level: row pairs -> carried bins (natural order) of `rows`
// rows, column-major into fft_b (bin k of row r at k * rows + r, the layout
// the y phase transforms).  Source: the round's aggregated component lists,
// or (KSRC) the PSF kernel image.
template <typename PT, bool KSRC, bool BIG = false>
__device__ void xfwd_one(const KArgs &a, const FftAxis &fx, int Ly, int rows, const int32_t *s_off, float2 *lds,
                         int *s_nz)
{
    const int Lx = fx.L, lgx = fx.lg, nx = a.nx, tx = a.tx;
    // LDS slot of transform element i (the wide-tile kernel's arena is padded)
    auto at = [](int i) { return pad16(i); };
    Tw13 T13;
    if (BIG && lgx == F13) tw13_load(T13, fx.tw);
    const int npr = (rows + 1) / 2;
    #pragma clang loop unroll(disable)
    for (int pr = xcd_slot(); pr < npr; pr += gridDim.x) {
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < rows;
        if (KSRC) {
            #pragma clang loop unroll(disable)
            for (int x = threadIdx.x; x < Lx; x += WG)
                lds[at(bitrev((uint32_t)x, lgx))] = make_float2(kernel_value<PT>(a, Ly, Lx, r0, x),
                                                                has1 ? kernel_value<PT>(a, Ly, Lx, r0 + 1, x) : 0.0f);
            if (threadIdx.x == 0) *s_nz = 1;
            __syncthreads();
        } else {
            const int slots = fft_pad_slots(Lx);
            #pragma clang loop unroll(disable)
            for (int x = threadIdx.x; x < slots; x += WG) lds[x] = make_float2(0.f, 0.f);
            if (threadIdx.x == 0) *s_nz = 0;
            __syncthreads();
            // the components of the two rows: the aggregated list of every
            // tile a row crosses is scanned by G threads, eight entries per
            // thread in flight (positions are distinct, so no two threads
            // write one slot)
            const int G = max(1, WG / (2 * tx));
            const int tr0 = tile_row_of(a, r0), tr1 = has1 ? tile_row_of(a, r0 + 1) : tr0;
            #pragma clang loop unroll(disable)
            for (int j = threadIdx.x; j < 2 * tx * G; j += WG) {
                const int part = j / (tx * G);           // 0: row r0 (real part), 1: row r0 + 1
                const int row = r0 + part;
                if (row >= rows) continue;
                const int t = (part ? tr1 : tr0) * tx + (j / G) % tx, q = j % G;
                const int n = s_off[t + 1] - s_off[t];
                const int32_t b0 = row * nx;
                const size_t base = (size_t)t * a.interval;
                int cnt = 0;
                #pragma clang loop unroll(disable)
                for (int e0 = q; e0 < n; e0 += 8 * G) {
                    int32_t pos[8];
                    float fl[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int e = e0 + u * G;
                        pos[u] = e < n ? ldc(&a.ag_pos[base + e]) : -1;
                        fl[u] = e < n ? ldc(&a.ag_flux[base + e]) : 0.0f;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (pos[u] >= b0 && pos[u] < b0 + nx) {
                            ((float *)&lds[at(bitrev((uint32_t)(pos[u] - b0), lgx))])[part] = fl[u];
                            ++cnt;
                        }
                }
                if (cnt) atomicAdd(s_nz, cnt);
            }
            __syncthreads();
        }
        float2 *o = a.fft_b + r0;
        if (*s_nz == 0) {                       // both rows empty: zero spectra
            #pragma clang loop unroll(disable)
            for (int k = threadIdx.x; k < fx.H; k += WG) store_cols(o, rows, has1, k, make_float2(0.f, 0.f),
                                                                   make_float2(0.f, 0.f));
        } else {
            if constexpr (BIG) {
                if (lgx == F13) fft13<false, false>(lds, T13);
                else fft_big<false>(lds, lgx, fx.tw, false);
            } else {
                fft_lds(lds, lgx, fx.tw, false);
            }
            #pragma clang loop unroll(disable)
            for (int k = threadIdx.x; k < fx.H; k += WG)
                store_cols(o, rows, has1, k, lds[at(k)], lds[at((Lx - k) & (Lx - 1))]);
        }
        __syncthreads();
    }
}

// x forward, two levels, step 1: per row pair and n2, transforms of length L1
// over n1 (input x = L2 n1 + n2), times W_L^(n2 k1), into fft_wx[pair][L2 k1 + n2].
// Source: the dense component image, or (KSRC) the PSF kernel image.
template <typename PT, bool KSRC, int U = STAGE_TWO>
__device__ __forceinline__ void xfwd_two_a(const KArgs &a, const FftAxis &fx, int Ly, int rows, float2 *lds)
{
    const int lgNB = strided_block_lg(fx), NB = 1 << lgNB;
    const int nblk = fx.L2 / NB, stride = fft_seg_stride(fx.L1);
    const int ncols = KSRC ? fx.L : a.nx;
    #pragma clang loop unroll(disable)
    for (int item = blockIdx.x; item < (rows + 1) / 2 * nblk; item += gridDim.x) {
        const int pr = item / nblk, b = item % nblk;
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < rows;
        staged<U>(NB * fx.L1, true,
                  [&](int e) {
                      const int x = fx.L2 * (e >> lgNB) + b * NB + (e & (NB - 1));
                      float v0 = 0.f, v1 = 0.f;
                      if (KSRC) {                          // once per call
                          if (x < ncols) {
                              v0 = kernel_value<PT>(a, Ly, fx.L, r0, x);
                              if (has1) v1 = kernel_value<PT>(a, Ly, fx.L, r0 + 1, x);
                          }
                      } else {                             // column clamped; zeroed in the write
                          const int xc = min(x, ncols - 1);
                          v0 = ldc(&a.comp_img[(size_t)r0 * a.nx + xc]);
                          v1 = ldc(&a.comp_img[(size_t)(has1 ? r0 + 1 : r0) * a.nx + xc]);
                      }
                      return make_float2(v0, v1);
                  },
                  [&](int e, float2 v) {
                      const int x = fx.L2 * (e >> lgNB) + b * NB + (e & (NB - 1));
                      if (!KSRC) v = x < ncols ? make_float2(v.x, has1 ? v.y : 0.f) : make_float2(0.f, 0.f);
                      lds[(e & (NB - 1)) * stride + pad16(bitrev((uint32_t)(e >> lgNB), fx.lg1))] = v;
                  });
        fft_lds_multi(lds, fx.lg1, NB, stride, fx.tw, fx.L2, false);
        float2 *w = a.fft_wx + (size_t)pr * fx.L;
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < NB * fx.L1; e += WG) {
            const int j = e & (NB - 1), k1 = e >> lgNB, n2 = b * NB + j;
            stc2(&w[(size_t)fx.L2 * k1 + n2], cmul(lds[j * stride + pad16(k1)], fx.tw[n2 * k1]));
        }
    }
}

// x forward, two levels, step 2: per row pair, rows k1 and L1 - k1 of the
// step-1 output transformed over n2 (length L2), then split into the two
// image rows' carried bins (chat order), column-major into fft_b like
// xfwd_one.  Unless KSRC, also clears the dense component image at this
// round's positions.
template <bool KSRC, int U = STAGE_TWO>
__device__ __forceinline__ void xfwd_two_b(const KArgs &a, const FftAxis &fx, int rows, float2 *lds, const int32_t *s_off)
{
    const int nslot = fx.L1 / 2 + 1;
    const int stride = fft_seg_stride(fx.L2);
    const int G = max(1, min(nslot, FFT_LDS_CPLX / (2 * stride)));
    const int nblk = (nslot + G - 1) / G;
    const int hq = fx.L2 / 2;
    const int npr = (rows + 1) / 2;
    // items (slot block, row pair) with the row pair fastest: the workgroups
    // of one XCD take consecutive row pairs of one block (xcd_slot)
    #pragma clang loop unroll(disable)
    for (int item = xcd_slot(); item < npr * nblk; item += gridDim.x) {
        const int pr = item % npr, s0 = (item / npr) * G, ns = min(G, nslot - s0);
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < rows;
        const float2 *w = a.fft_wx + (size_t)pr * fx.L;
        // segment 2i: row k1 = s0 + i; segment 2i+1: row (L1 - k1) mod L1
        staged<U>(2 * ns * fx.L2, true,
                  [&](int e) {
                      const int seg = e >> fx.lg2, n2 = e & (fx.L2 - 1);
                      const int k1 = s0 + (seg >> 1);
                      const int kr = (seg & 1) ? ((fx.L1 - k1) & (fx.L1 - 1)) : k1;
                      return ldc2(&w[(size_t)fx.L2 * kr + n2]);
                  },
                  [&](int e, float2 v) { lds[(e >> fx.lg2) * stride + pad16(bitrev((uint32_t)(e & (fx.L2 - 1)), fx.lg2))] = v; });
        fft_lds_multi(lds, fx.lg2, 2 * ns, stride, fx.tw, fx.L1, false);
        float2 *o = a.fft_b + r0;
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < 2 * ns * hq; e += WG) {
            const int seg = e >> (fx.lg2 - 1), k2 = e & (hq - 1);
            const int k1 = s0 + (seg >> 1);
            const bool second = seg & 1;
            if (second && (k1 == 0 || 2 * k1 == fx.L1)) continue;      // row is its own mirror
            const int kr = second ? fx.L1 - k1 : k1;
            int q1, q2;
            mirror_of(fx, kr, k2, q1, q2);
            const int qs = q1 == kr ? seg : (seg ^ 1);
            store_cols(o, rows, has1, chat_of(fx, kr, k2), lds[seg * stride + pad16(k2)], lds[qs * stride + pad16(q2)]);
        }
        if (s0 == 0 && threadIdx.x == 0)        // bin k = L/2: row 0, k2 = L2/2, its own mirror
            store_cols(o, rows, has1, fx.L / 2, lds[pad16(hq)], lds[pad16(hq)]);
    }
    if (!KSRC) {
        const int total = s_off[a.T];
        #pragma clang loop unroll(disable)
        for (int i = blockIdx.x * WG + threadIdx.x; i < total; i += gridDim.x * WG) {
            int lo = 0, hi = a.T;                   // largest t with s_off[t] <= i
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= i) lo = mid; else hi = mid;
            }
            stc(&a.comp_img[ldc(&a.ag_pos[(size_t)lo * a.interval + (i - s_off[lo])])], 0.0f);
        }
    }
}

// y, one level, per carried column: forward transform of the `rows` values
// in fft_b; then either (PRE) store the spectrum as the PSF kernel's, or
// multiply by it, transform back and store the first `rows` values.
// The wide-tile kernel's y phase at length 8192, per carried column: the
// column and its zero padding (natural order) -> forward in frequency order
// -> product with the PSF kernel's spectrum (held in the same bit-reversed
// order) -> inverse in time order -> the first `rows` values.  Fused where
// the data allow: the forward's first pass takes the column from registers,
// the forward's last stage, the product and the inverse's first stage are one
// sweep over the pairs (2j, 2j+1), and the inverse's last pass leaves the
// result in registers for the stores.  The next column's values and spectrum
// are loaded while this one is transformed.
__device__ void ycol13(const KArgs &a, const FftAxis &fx, int rows, float2 *lds)
{
    constexpr int L = 1 << F13, M = L / WG;
    Tw13 T;
    tw13_load(T, a.tw_y);
    const int t = threadIdx.x;
    float2 nb[M];                   // the column, elements t + WG m
    float4 nk[M / 2];               // the spectrum at slots 2j, 2j+1 of j = t + WG m
    auto load_b = [&](int c) {
        const float2 *b = a.fft_b + (size_t)c * rows;
#pragma unroll
        for (int m = 0; m < M; ++m) nb[m] = ldc2(b + min(t + WG * m, rows - 1));
    };
    auto load_k = [&](int c) {
        const float2 *k = a.fft_ks + (size_t)c * L;
#pragma unroll
        for (int m = 0; m < M / 2; ++m) {
            const float2 k0 = ldc2(k + 2 * t + 2 * WG * m), k1 = ldc2(k + 2 * t + 2 * WG * m + 1);
            nk[m] = make_float4(k0.x, k0.y, k1.x, k1.y);
        }
    };
    float2 *const b9 = f13_base<9>(lds);            // element t + WG m at b9[pad16c(WG m)]
    float2 *const p2 = lds + pad16(2 * t);           // pair j = t + WG m at p2[pad16c(2 WG m)], +1
    int col = blockIdx.x;
    if (col < fx.H) {
        load_b(col);
        load_k(col);
    }
    #pragma clang loop unroll(disable)
    for (; col < fx.H; col += gridDim.x) {
        const int nxt = col + gridDim.x;
        float2 x[M];
#pragma unroll
        for (int m = 0; m < M; ++m) x[m] = t + WG * m < rows ? nb[m] : make_float2(0.f, 0.f);
        if (nxt < fx.H) load_b(nxt);
        f13_units<9, true, false>(x, T.w[2]);
        __syncthreads();                            // the previous column's last reads are done
#pragma unroll
        for (int m = 0; m < M; ++m) b9[pad16c(WG * m)] = x[m];
        __syncthreads();
        f13_pass16<5, true, false>(lds, T.w[1]);
        f13_pass16<1, true, false>(lds, T.w[0]);
#pragma unroll
        for (int m = 0; m < M / 2; ++m) {
            float2 *q = p2 + pad16c(2 * WG * m);
            const float2 u = q[0], v = q[1];
            const float2 f0 = twmul<false>(make_float2(u.x + v.x, u.y + v.y), make_float2(nk[m].x, nk[m].y));
            const float2 f1 = twmul<false>(make_float2(u.x - v.x, u.y - v.y), make_float2(nk[m].z, nk[m].w));
            q[0] = make_float2(f0.x + f1.x, f0.y + f1.y);
            q[1] = make_float2(f0.x - f1.x, f0.y - f1.y);
        }
        __syncthreads();
        if (nxt < fx.H) load_k(nxt);
        f13_pass16<1, false, true>(lds, T.w[0]);
        f13_pass16<5, false, true>(lds, T.w[1]);
#pragma unroll
        for (int m = 0; m < M; ++m) x[m] = b9[pad16c(WG * m)];
        f13_units<9, false, true>(x, T.w[2]);
        float2 *b = a.fft_b + (size_t)col * rows;
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (t + WG * m < rows) stc2(b + t + WG * m, x[m]);
    }
}

template <bool PRE, bool BIG = false>
__device__ void ycol_one(const KArgs &a, const FftAxis &fx, const FftAxis &fy, int rows, float2 *lds)
{
    if constexpr (BIG && !PRE) {
        if (fy.lg == F13) {
            ycol13(a, fx, rows, lds);
            return;
        }
    }
    #pragma clang loop unroll(disable)
    for (int col = blockIdx.x; col < fx.H; col += gridDim.x) {
        float2 *b = a.fft_b + (size_t)col * rows;
        float2 *ks = a.fft_ks + (size_t)col * fy.L;
        if constexpr (BIG) {
            // padded arena, no permutation: the column and its zero padding in
            // natural order, forward in frequency order (bit-reversed spectrum,
            // the PSF kernel's spectrum stored in the same order), product,
            // inverse in time order (natural output)
            staged<16>(fy.L, true, [&](int v) { return ldc2(&b[min(v, rows - 1)]); },
                       [&](int v, float2 z) { lds[pad16(v)] = v < rows ? z : make_float2(0.f, 0.f); });
            if (fy.lg == F13) {
                Tw13 T;
                tw13_load(T, fy.tw);
                fft13<true, false>(lds, T);
            } else {
                fft_big<true>(lds, fy.lg, fy.tw, false);
            }
            if (PRE) {
                #pragma clang loop unroll(disable)
                for (int v = threadIdx.x; v < fy.L; v += WG) stc2(&ks[v], lds[pad16(v)]);
            } else {
                staged<16>(fy.L, false, [&](int v) { return ldc2(&ks[v]); },
                           [&](int v, float2 k) { lds[pad16(v)] = cmul(lds[pad16(v)], k); });
                fft_big<false>(lds, fy.lg, fy.tw, true);
                #pragma clang loop unroll(disable)
                for (int v = threadIdx.x; v < rows; v += WG) stc2(&b[v], lds[pad16(v)]);
            }
        } else {
            #pragma clang loop unroll(disable)
            for (int v = threadIdx.x; v < fft_pad_slots(fy.L); v += WG) lds[v] = make_float2(0.f, 0.f);
            __syncthreads();
            #pragma clang loop unroll(disable)
            for (int v = threadIdx.x; v < rows; v += WG) lds[pad16(bitrev((uint32_t)v, fy.lg))] = ldc2(&b[v]);
            fft_lds(lds, fy.lg, fy.tw, false);
            if (PRE) {
                #pragma clang loop unroll(disable)
                for (int v = threadIdx.x; v < fy.L; v += WG) stc2(&ks[v], lds[pad16(v)]);
            } else {
                #pragma clang loop unroll(disable)
                for (int v = threadIdx.x; v < fy.L; v += WG) lds[pad16(v)] = cmul(lds[pad16(v)], ldc2(&ks[v]));
                bitrev_permute(lds, fy.lg);
                fft_lds(lds, fy.lg, fy.tw, true);
                #pragma clang loop unroll(disable)
                for (int v = threadIdx.x; v < rows; v += WG) stc2(&b[v], lds[pad16(v)]);
            }
        }
        __syncthreads();
    }
}

// y, two levels, step 1: per carried column and n2, transforms of length L1
// over n1 (input y = L2 n1 + n2 < rows), times W_L^(n2 k1), into
// fft_wy[col][L2 k1 + n2].
template <int U = STAGE_TWO>
__device__ __forceinline__ void ycol_two_a(const KArgs &a, const FftAxis &fx, const FftAxis &fy, int rows, float2 *lds)
{
    const int lgNB = strided_block_lg(fy), NB = 1 << lgNB;
    const int nblk = fy.L2 / NB, stride = fft_seg_stride(fy.L1);
    #pragma clang loop unroll(disable)
    for (int item = blockIdx.x; item < fx.H * nblk; item += gridDim.x) {
        const int col = item / nblk, b = item % nblk;
        const float2 *src = a.fft_b + (size_t)col * rows;
        staged<U>(NB * fy.L1, true,
                  [&](int e) { return ldc2(&src[min(fy.L2 * (e >> lgNB) + b * NB + (e & (NB - 1)), rows - 1)]); },
                  [&](int e, float2 v) {
                      const int yy = fy.L2 * (e >> lgNB) + b * NB + (e & (NB - 1));
                      lds[(e & (NB - 1)) * stride + pad16(bitrev((uint32_t)(e >> lgNB), fy.lg1))] =
                          yy < rows ? v : make_float2(0.f, 0.f);
                  });
        fft_lds_multi(lds, fy.lg1, NB, stride, fy.tw, fy.L2, false);
        float2 *w = a.fft_wy + (size_t)col * fy.L;
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < NB * fy.L1; e += WG) {
            const int j = e & (NB - 1), k1 = e >> lgNB, n2 = b * NB + j;
            stc2(&w[(size_t)fy.L2 * k1 + n2], cmul(lds[j * stride + pad16(k1)], fy.tw[n2 * k1]));
        }
    }
}

// y, two levels, step 2: per carried column and row k1 of the step-1 output,
// transform over n2 (length L2, frequency order); then either (PRE) store as
// the PSF kernel's spectrum in (k1, bit-reversed k2) order, or multiply by it,
// transform back over k2 (time order: no permutation between), times
// conj W_L^(n2 k1), into fft_wy.
template <bool PRE, int U = STAGE_TWO>
__device__ __forceinline__ void ycol_two_b(const KArgs &a, const FftAxis &fx, const FftAxis &fy, float2 *lds)
{
    const int stride = fft_seg_stride(fy.L2);
    const int G = max(1, min(fy.L1, FFT_LDS_CPLX / stride));
    const int nblk = (fy.L1 + G - 1) / G;
    #pragma clang loop unroll(disable)
    for (int item = blockIdx.x; item < fx.H * nblk; item += gridDim.x) {
        const int col = item / nblk, k0 = (item % nblk) * G, ng = min(G, fy.L1 - k0);
        float2 *w = a.fft_wy + (size_t)col * fy.L;
        float2 *ks = a.fft_ks + (size_t)col * fy.L;
        // natural order in, forward in frequency order: the spectrum (and the
        // PSF kernel's, made by the same code) in bit-reversed k2 order, which
        // the inverse below takes as it is
        staged<U>(ng * fy.L2, true,
                  [&](int e) { return ldc2(&w[(size_t)fy.L2 * (k0 + (e >> fy.lg2)) + (e & (fy.L2 - 1))]); },
                  [&](int e, float2 v) { lds[(e >> fy.lg2) * stride + pad16(e & (fy.L2 - 1))] = v; });
        fft_lds_multi_dif(lds, fy.lg2, ng, stride, fy.tw, fy.L1, false);
        if (PRE) {
            #pragma clang loop unroll(disable)
            for (int e = threadIdx.x; e < ng * fy.L2; e += WG) {
                const int g = e >> fy.lg2, k2 = e & (fy.L2 - 1);
                stc2(&ks[(size_t)fy.L2 * (k0 + g) + k2], lds[g * stride + pad16(k2)]);
            }
            continue;
        }
        staged<U>(ng * fy.L2, false,
                  [&](int e) { return ldc2(&ks[(size_t)fy.L2 * (k0 + (e >> fy.lg2)) + (e & (fy.L2 - 1))]); },
                  [&](int e, float2 k) {
                      float2 &z = lds[(e >> fy.lg2) * stride + pad16(e & (fy.L2 - 1))];
                      z = cmul(z, k);
                  });
        fft_lds_multi(lds, fy.lg2, ng, stride, fy.tw, fy.L1, true);
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < ng * fy.L2; e += WG) {
            const int g = e >> fy.lg2, n2 = e & (fy.L2 - 1), k1 = k0 + g;
            stc2(&w[(size_t)fy.L2 * k1 + n2], cmulc(lds[g * stride + pad16(n2)], fy.tw[n2 * k1]));
        }
    }
}

// y, two levels, step 3: per carried column and n2, inverse transforms of
// length L1 over k1, giving y = L2 n1 + n2; the first `rows` go to fft_b.
template <int U = STAGE_TWO>
__device__ __forceinline__ void ycol_two_c(const KArgs &a, const FftAxis &fx, const FftAxis &fy, int rows, float2 *lds)
{
    const int lgNB = strided_block_lg(fy), NB = 1 << lgNB;
    const int nblk = fy.L2 / NB, stride = fft_seg_stride(fy.L1);
    #pragma clang loop unroll(disable)
    for (int item = blockIdx.x; item < fx.H * nblk; item += gridDim.x) {
        const int col = item / nblk, b = item % nblk;
        const float2 *w = a.fft_wy + (size_t)col * fy.L;
        staged<U>(NB * fy.L1, true,
                  [&](int e) { return ldc2(&w[(size_t)fy.L2 * (e >> lgNB) + b * NB + (e & (NB - 1))]); },
                  [&](int e, float2 v) { lds[(e & (NB - 1)) * stride + pad16(bitrev((uint32_t)(e >> lgNB), fy.lg1))] = v; });
        fft_lds_multi(lds, fy.lg1, NB, stride, fy.tw, fy.L2, true);
        float2 *dst = a.fft_b + (size_t)col * rows;
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < NB * fy.L1; e += WG) {
            const int j = e & (NB - 1), n1 = e >> lgNB;
            const int yy = fy.L2 * n1 + b * NB + j;
            if (yy < rows) stc2(&dst[yy], lds[j * stride + pad16(n1)]);
        }
    }
}

// The wide-tile kernel's x inverse at length 8192 (the steps of xinv_one):
// the next row pair's carried bins are loaded while this one is transformed.
__device__ void xinv13(const KArgs &a, const FftAxis &fx, float scale, float2 *lds)
{
    constexpr int L = 1 << F13, H = L / 2 + 1, M = (H + WG - 1) / WG;
    Tw13 T;
    tw13_load(T, a.tw_x);
    const int t = threadIdx.x, ny = a.ny, nx = a.nx, npr = (ny + 1) / 2;
    float2 nA[M], nB[M];
    auto load = [&](int pr) {
        const float2 *c0 = a.fft_b + 2 * pr;
        const bool has1 = 2 * pr + 1 < ny;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = t + WG * m, kc = min(k, H - 1);
            float2 A, B = make_float2(0.f, 0.f);
            if ((ny & 1) == 0) {
                const f32x4 q = ldp4(c0 + (size_t)kc * ny);
                A = make_float2(q.x, q.y);
                B = make_float2(q.z, q.w);
            } else {
                A = ldp2(c0 + (size_t)kc * ny);
                if (has1) B = ldp2(c0 + (size_t)kc * ny + 1);
            }
            nA[m] = k < H ? A : make_float2(0.f, 0.f);
            nB[m] = k < H ? B : make_float2(0.f, 0.f);
        }
    };
    int pr = xcd_slot();
    if (pr < npr) load(pr);
    #pragma clang loop unroll(disable)
    for (; pr < npr; pr += gridDim.x) {
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < ny;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int k = t + WG * m;
            if (k < H) {
                const float2 A = nA[m], B = nB[m];
                lds[pad16(bitrev((uint32_t)k, F13))] = make_float2(A.x - B.y, A.y + B.x);
                if (k > 0 && k < L / 2) lds[pad16(bitrev((uint32_t)(L - k), F13))] = make_float2(A.x + B.y, B.x - A.y);
            }
        }
        if (pr + (int)gridDim.x < npr) load(pr + gridDim.x);
        fft13<false, true>(lds, T);
        #pragma clang loop unroll(disable)
        for (int x = t; x < nx; x += WG) {
            const float2 z = lds[pad16(x)];
            stc(&a.accbuf[(size_t)r0 * nx + x], z.x * scale);
            if (has1) stc(&a.accbuf[(size_t)(r0 + 1) * nx + x], z.y * scale);
        }
    }
}

// x inverse, one level: row pairs rebuilt from their carried bins (Hermitian
// symmetry gives the rest; read column-major from fft_b, where the y phase
// leaves them), one inverse transform, real part -> row 2m, imaginary part ->
// row 2m+1, scaled, into the feedback buffer.
template <bool BIG = false>
__device__ void xinv_one(const KArgs &a, const FftAxis &fx, float scale, float2 *lds)
{
    if constexpr (BIG) {
        if (fx.lg == F13) {
            xinv13(a, fx, scale, lds);
            return;
        }
    }
    const int Lx = fx.L, lgx = fx.lg, ny = a.ny, nx = a.nx;
    auto at = [](int i) { return pad16(i); };
    #pragma clang loop unroll(disable)
    for (int pr = xcd_slot(); pr < (ny + 1) / 2; pr += gridDim.x) {
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < ny;
        const float2 *c0 = a.fft_b + r0;
        #pragma clang loop unroll(disable)
        for (int k = threadIdx.x; k < fx.H; k += WG) {
            float2 A, B = make_float2(0.f, 0.f);
            if ((ny & 1) == 0) {
                const f32x4 q = ldp4(c0 + (size_t)k * ny);
                A = make_float2(q.x, q.y);
                B = make_float2(q.z, q.w);
            } else {
                A = ldp2(c0 + (size_t)k * ny);
                if (has1) B = ldp2(c0 + (size_t)k * ny + 1);
            }
            lds[at(bitrev((uint32_t)k, lgx))] = make_float2(A.x - B.y, A.y + B.x);
            if (k > 0 && k < Lx / 2) lds[at(bitrev((uint32_t)(Lx - k), lgx))] = make_float2(A.x + B.y, B.x - A.y);
        }
        if constexpr (BIG) fft_big<false>(lds, lgx, fx.tw, true);
        else fft_lds(lds, lgx, fx.tw, true);
        #pragma clang loop unroll(disable)
        for (int x = threadIdx.x; x < nx; x += WG) {
            const float2 z = lds[at(x)];
            stc(&a.accbuf[(size_t)r0 * nx + x], z.x * scale);
            if (has1) stc(&a.accbuf[(size_t)(r0 + 1) * nx + x], z.y * scale);
        }
        __syncthreads();
    }
}

// x inverse, two levels, step 1: per row pair and row k1, Z(k1, k2) for all
// k2 from the carried bins (A + iB, or conj A + i conj B at mirrored bins),
// inverse transform over k2 (length L2), times conj W_L^(n2 k1), into fft_wx.
template <int U = STAGE_TWO>
__device__ __forceinline__ void xinv_two_a(const KArgs &a, const FftAxis &fx, float2 *lds)
{
    const int ny = a.ny, stride = fft_seg_stride(fx.L2), hq = fx.L2 / 2;
    const int G = max(1, min(fx.L1, FFT_LDS_CPLX / stride));
    const int nblk = (fx.L1 + G - 1) / G;
    const int npr = (ny + 1) / 2;
    // items (row block, row pair) with the row pair fastest, as in xfwd_two_b
    #pragma clang loop unroll(disable)
    for (int item = xcd_slot(); item < npr * nblk; item += gridDim.x) {
        const int pr = item % npr, k0 = (item / npr) * G, ng = min(G, fx.L1 - k0);
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < ny;
        const float2 *c0 = a.fft_b + r0;       // bin c of the pair at c0[c * ny], c0[c * ny + 1]
        staged<U>(ng * fx.L2, true,
                  [&](int e) {
                      const int k2 = e & (fx.L2 - 1), k1 = k0 + (e >> fx.lg2);
                      const bool carried = k2 < hq || (k2 == hq && k1 == 0);
                      int q1 = k1, q2 = k2;
                      if (!carried) mirror_of(fx, k1, k2, q1, q2);
                      const float2 *p = c0 + (size_t)chat_of(fx, q1, q2) * ny;
                      if ((ny & 1) == 0) {
                          const f32x4 q = ldp4(p);
                          return make_float4(q.x, q.y, q.z, q.w);
                      }
                      const float2 A = ldp2(p), B = ldp2(has1 ? p + 1 : p);   // B unused without row r0 + 1
                      return make_float4(A.x, A.y, B.x, B.y);
                  },
                  [&](int e, float4 q) {
                      const int k2 = e & (fx.L2 - 1), k1 = k0 + (e >> fx.lg2);
                      const bool carried = k2 < hq || (k2 == hq && k1 == 0);
                      const float2 A = make_float2(q.x, q.y), B = has1 ? make_float2(q.z, q.w) : make_float2(0.f, 0.f);
                      lds[(e >> fx.lg2) * stride + pad16(bitrev((uint32_t)k2, fx.lg2))] =
                          carried ? make_float2(A.x - B.y, A.y + B.x) : make_float2(A.x + B.y, B.x - A.y);
                  });
        fft_lds_multi(lds, fx.lg2, ng, stride, fx.tw, fx.L1, true);
        float2 *w = a.fft_wx + (size_t)pr * fx.L;
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < ng * fx.L2; e += WG) {
            const int g = e >> fx.lg2, n2 = e & (fx.L2 - 1), k1 = k0 + g;
            stc2(&w[(size_t)fx.L2 * k1 + n2], cmulc(lds[g * stride + pad16(n2)], fx.tw[n2 * k1]));
        }
    }
}

// x inverse, two levels, step 2: per row pair and n2, inverse transforms of
// length L1 over k1 giving x = L2 n1 + n2; real / imaginary parts of the
// first nx, scaled, into the feedback buffer rows 2m / 2m+1.
template <int U = STAGE_TWO>
__device__ __forceinline__ void xinv_two_b(const KArgs &a, const FftAxis &fx, float scale, float2 *lds)
{
    const int ny = a.ny, nx = a.nx;
    const int lgNB = strided_block_lg(fx), NB = 1 << lgNB;
    const int nblk = fx.L2 / NB, stride = fft_seg_stride(fx.L1);
    #pragma clang loop unroll(disable)
    for (int item = blockIdx.x; item < (ny + 1) / 2 * nblk; item += gridDim.x) {
        const int pr = item / nblk, b = item % nblk;
        const int r0 = 2 * pr;
        const bool has1 = r0 + 1 < ny;
        const float2 *w = a.fft_wx + (size_t)pr * fx.L;
        staged<U>(NB * fx.L1, true,
                  [&](int e) { return ldc2(&w[(size_t)fx.L2 * (e >> lgNB) + b * NB + (e & (NB - 1))]); },
                  [&](int e, float2 v) { lds[(e & (NB - 1)) * stride + pad16(bitrev((uint32_t)(e >> lgNB), fx.lg1))] = v; });
        fft_lds_multi(lds, fx.lg1, NB, stride, fx.tw, fx.L2, true);
        #pragma clang loop unroll(disable)
        for (int e = threadIdx.x; e < NB * fx.L1; e += WG) {
            const int j = e & (NB - 1), n1 = e >> lgNB;
            const int x = fx.L2 * n1 + b * NB + j;
            if (x < nx) {
                const float2 z = lds[j * stride + pad16(n1)];
                stc(&a.accbuf[(size_t)r0 * nx + x], z.x * scale);
                if (has1) stc(&a.accbuf[(size_t)(r0 + 1) * nx + x], z.y * scale);
            }
        }
    }
}

#define FFT_BARRIER() do { if (!xcd_grid_barrier(y, xb, s_ok)) return false; } while (0)
#define FFT_BARRIER_FENCED() do { if (!xcd_grid_barrier<true>(y, xb, s_ok)) return false; } while (0)

// The PSF kernel's spectrum, once per call, by the same transforms as the
// rounds: x forward over all Ly rows of the kernel image, y forward.  A
// function of its own (called once per launch), its arguments by value or by
// address, so that none of them needs a stack copy.
template <typename PT, bool BIG = false>
__device__ __noinline__ bool fft_spectrum(const KArgs *a_arg, const Sync y_arg, XcdBar *xb_arg, int *s_ok)
{
    const KArgs &a = *wave_uniform(a_arg);
    const Sync y = wave_uniform(y_arg);
    XcdBar *xb = wave_uniform(xb_arg);
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ int s_nz;
    float2 *lds = (float2 *)s_dyn;
    const FftAxis fx = fft_axis(a.fft_lgx, a.fft_two_x, a.tw_x), fy = fft_axis(a.fft_lgy, a.fft_two_y, a.tw_y);
    const int Ly = fy.L;
    if (!fx.two) {
        xfwd_one<PT, true, BIG>(a, fx, Ly, Ly, nullptr, lds, &s_nz);
    } else {
        xfwd_two_a<PT, true, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, Ly, Ly, lds);
        FFT_BARRIER();
        xfwd_two_b<true, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, Ly, lds, nullptr);
    }
    FFT_BARRIER_FENCED();
    if (!fy.two) {
        ycol_one<true, BIG>(a, fx, fy, Ly, lds);
    } else {
        ycol_two_a<BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy, Ly, lds);
        FFT_BARRIER();
        ycol_two_b<true, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy, lds);
    }
    FFT_BARRIER();
    return true;
}

// One round's feedback sums: the component image (*) the PSF, every tile's
// components, own tile included, into the feedback buffer.  The apply step
// then recomputes the residual from the round's starting residual:
// mathematically the paper's update (own components subtracted locally, the
// others' by feedback), rounded once.  The x phases write and read the y
// phase's column-major layout directly; fenced barriers separate them from it.
template <typename PT, bool BIG = false>
__device__ __forceinline__ bool fft_feedback(const KArgs &a, const Sync &y, XcdBar *xb, int *s_ok, const int32_t *s_off)
{
    extern __shared__ __align__(16) unsigned char s_dyn[];
    __shared__ int s_nz;
    float2 *lds = (float2 *)s_dyn;
    const FftAxis fx = fft_axis(a.fft_lgx, a.fft_two_x, a.tw_x), fy = fft_axis(a.fft_lgy, a.fft_two_y, a.tw_y);
    const int ny = a.ny;
    const float scale = 1.0f / ((float)fx.L * (float)fy.L);
    if (!fx.two) {
        xfwd_one<PT, false, BIG>(a, fx, fy.L, ny, s_off, lds, &s_nz);
    } else {
        xfwd_two_a<PT, false, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy.L, ny, lds);
        FFT_BARRIER();
        xfwd_two_b<false, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, ny, lds, s_off);
    }
    FFT_BARRIER_FENCED();
    if (!fy.two) {
        ycol_one<false, BIG>(a, fx, fy, ny, lds);
    } else {
        ycol_two_a<BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy, ny, lds);
        FFT_BARRIER();
        ycol_two_b<false, BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy, lds);
        FFT_BARRIER();
        ycol_two_c<BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, fy, ny, lds);
    }
    FFT_BARRIER_FENCED();
    if (!fx.two) {
        xinv_one<BIG>(a, fx, scale, lds);
    } else {
        xinv_two_a<BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, lds);
        FFT_BARRIER();
        xinv_two_b<BIG ? STAGE_TWO_WIDE : STAGE_TWO>(a, fx, scale, lds);
    }
    __syncthreads();
    return true;
}

// The wide-tile kernel's feedback round in a function of its own: its
// transform loops get a register allocation of their own, unaffected by the
// state the round loop keeps live (inlined, that state pushed spills into the
// transform passes).  Arguments are copied to scalar registers first: the
// argument block's address and the wait settings are the same in every lane.
template <typename PT>
__device__ __noinline__ bool fft_feedback_wide(const KArgs *a_arg, const Sync y_arg, XcdBar *xb_arg, int *s_ok,
                                               const int32_t *s_off)
{
    const KArgs *ap = wave_uniform(a_arg);
    const Sync y = wave_uniform(y_arg);
    XcdBar *xb = wave_uniform(xb_arg);
    return fft_feedback<PT, true>(*ap, y, xb, s_ok, s_off);
}

#undef FFT_BARRIER
#undef FFT_BARRIER_FENCED

// ------------------------------------------------------ tiled kernel -----

// Aggregate the leader's round list (LDS) by position: distinct positions in
// ascending order, each with the float64 sum of its components in the order
// found, rounded once to float32; zero sums are dropped.  Writes the raw list
// and the aggregated list of tile t to global memory.  The four LDS arrays
// start on 16-byte boundaries; every scan reads the list four entries at a
// time and runs its full length (no early exit), so it is bound by LDS
// throughput, not by the latency of one read after another.
__device__ void aggregate_round(const KArgs &a, int t, int L, int32_t *l_idx, float *l_flux, int32_t *l_tmp,
                                float *l_sum, int *s_cnt)
{
    constexpr int32_t NONE = 0x7FFFFFFF;        // above every pixel index
    const size_t base = (size_t)t * a.interval;
    for (int j = threadIdx.x; j < L; j += WG) {
        stc(&a.rb_idx[base + j], l_idx[j]);
        stc(&a.rb_flux[base + j], l_flux[j]);
    }
    const int L4 = L & ~3;
    // pass 1: entry j is kept if no earlier entry has its position and the
    // float64 sum of the entries from j on with that position, in order, is
    // not zero; l_tmp[j] = its position if kept, else NONE
    for (int j = threadIdx.x; j < L; j += WG) {
        const int32_t q = l_idx[j];
        bool dup = false;
        double s = 0.0;
        for (int k = 0; k < L4; k += 4) {
            const int4 v = *(const int4 *)&l_idx[k];
            const int32_t vv[4] = {v.x, v.y, v.z, v.w};
            if ((vv[0] == q) | (vv[1] == q) | (vv[2] == q) | (vv[3] == q)) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (vv[e] == q) {
                        if (k + e < j) dup = true;
                        else s += (double)l_flux[k + e];
                    }
                }
            }
        }
        for (int k = L4; k < L; ++k) {
            if (l_idx[k] == q) {
                if (k < j) dup = true;
                else s += (double)l_flux[k];
            }
        }
        const bool keep = !dup && s != 0.0;
        l_tmp[j] = keep ? q : NONE;
        l_sum[j] = (float)s;
    }
    __syncthreads();
    // pass 2: rank of each kept position among the kept positions
    int mine = 0;
    for (int j = threadIdx.x; j < L; j += WG) {
        const int32_t q = l_tmp[j];
        if (q == NONE) continue;
        int rk = 0;
        for (int k = 0; k < L4; k += 4) {
            const int4 v = *(const int4 *)&l_tmp[k];
            rk += (v.x < q) + (v.y < q) + (v.z < q) + (v.w < q);
        }
        for (int k = L4; k < L; ++k) rk += l_tmp[k] < q;
        stc(&a.ag_pos[base + rk], q);
        stc(&a.ag_flux[base + rk], l_sum[j]);
        if (a.comp_img) stc(&a.comp_img[q], l_sum[j]);
        ++mine;
    }
    if (threadIdx.x == 0) *s_cnt = 0;
    __syncthreads();
    if (mine) atomicAdd(s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        stc(&a.rb_n[t], (int32_t)L);
        stc(&a.ag_n[t], (int32_t)*s_cnt);
    }
}

// Workgroup-wide sum of an int (every thread gets it).
__device__ __forceinline__ int wg_sum_int(int v, int *s_tmp)
{
    if (threadIdx.x == 0) *s_tmp = 0;
    __syncthreads();
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(s_tmp, v);
    __syncthreads();
    int r = *s_tmp;
    __syncthreads();
    return r;
}

// FFT selects the feedback form at compile time, so the direct-gather kernels
// carry none of the transform code (and its register needs).
// Streamed tiles with FFT feedback are capped at 128 VGPRs (four waves per
// SIMD) so that two workgroups share a CU, as the direct-gather ones do.
//
// tiled_body runs the rounds of one tiled problem on `members` workgroups,
// this one being member `member` with role `role` (tile << 16 | cluster rank,
// or -1: a helper of the feedback phases): the whole grid of tiled_kernel, or
// one problem's share of a batched launch (a.bar is then that problem's
// barrier counter and a.cword its cancel word).  xcd_items: spread the
// gather's items over the XCDs by workgroup index (the whole grid only).
template <class Tile, bool FFT, bool BATCH>
__device__ __forceinline__ void tiled_body(const KArgs &a, int member_arg, int members_arg, int32_t role, bool xcd_items)
{
    // the whole grid reads its index, size and control words from the
    // dispatch and the control block; a batched problem gets its own
    const int member = BATCH ? member_arg : (int)blockIdx.x;
    const int members = BATCH ? members_arg : (int)gridDim.x;
    constexpr int V = Tile::kV;
    using PT = typename Tile::psf_t;
    __shared__ int s_ok, s_tmp, s_cnt;
    __shared__ uint32_t s_vmax;
    __shared__ int32_t s_off[MAX_TILES + 1];    // exclusive prefix of per-tile counts
    extern __shared__ __align__(16) unsigned char s_dyn[];

    const Sync y{a.ctl, a.timeout_ticks};
    const Img im{a.dirty, a.residual, a.model, a.accbuf, a.rstart, a.psf, a.psf_bytes, a.nx, a.psf_nx, a.cy, a.cx};
    const bool is_cluster = role >= 0;
    const int tile = is_cluster ? (role >> 16) : -1;
    const int rank = is_cluster ? (role & 0xFFFF) : 0;
    const int cs = a.cs;
    const int T = a.T;
    uint64_t *slots = is_cluster ? a.xslots + (size_t)tile * 2 * a.slot_pad : nullptr;
    uint64_t *lslots = nullptr;     // set when the whole cluster shares one XCD
    const bool tile_leader_wg = is_cluster && rank == 0;

    // round-list LDS (leader workgroup) and gather staging (everyone) share s_dyn
    const size_t i4 = ((size_t)a.interval + 3) & ~(size_t)3;     // 16-byte aligned arrays
    int32_t *l_idx = (int32_t *)s_dyn;
    float *l_flux = (float *)(s_dyn + 4 * i4);
    int32_t *l_tmp = (int32_t *)(s_dyn + 8 * i4);
    float *l_sum = (float *)(s_dyn + 12 * i4);
    int32_t *g_shift = (int32_t *)s_dyn;
    float *g_flux = (float *)(s_dyn + 4 * (size_t)GATHER_CHUNK);

    Tile R;
    uint32_t e = 0, epoch = 0;
    uint64_t cur = 0;
    __shared__ XcdBar s_xb;
    if (!BATCH && threadIdx.x == 0) {
        s_xb = XcdBar{xcc_id(), 0, 0, 0};
        __hip_atomic_fetch_add(&a.ctl->xmem[s_xb.x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (is_cluster) {
        int ty0, tx0, th, tw;
        tile_rect(a, tile, ty0, tx0, th, tw);
        R.init(im, ty0, tx0, th, tw, cs, rank);
        if (!Tile::kResident) __syncthreads();
        uint64_t *ls = a.lslots + (size_t)tile * 2 * a.slot_pad;
        const int same = cluster_same_xcd(y, slots, ls, a.slot_pad, cs, rank, e++);
        if (same < 0) return;
        if (same) {
            lslots = ls;
            if (tile_leader_wg && threadIdx.x == 0)
                __hip_atomic_fetch_add(&a.dstat->xcd_local, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!cluster_reduce(y, slots, lslots, a.slot_pad, cs, rank, e++, R.key(im), cur)) return;
        if (tile_leader_wg && threadIdx.x == 0) stc(&a.tile_key[tile], cur);
        if constexpr (Tile::kWide && !BATCH) {
            // time-multiplexed clusters: the cluster's other tiles
            for (int t = tile + a.ncl; t < T; t += a.ncl) {
                int ty0, tx0, th, tw;
                tile_rect(a, t, ty0, tx0, th, tw);
                R.init(im, ty0, tx0, th, tw, cs, rank);
                __syncthreads();
                uint64_t k;
                if (!cluster_reduce(y, slots, lslots, a.slot_pad, cs, rank, e++, R.key(im), k)) return;
                if (tile_leader_wg && threadIdx.x == 0) stc(&a.tile_key[t], k);
            }
            if (a.ncl < T) R.init(im, ty0, tx0, th, tw, cs, rank, false);     // back to the first tile
        }
    }
    // the caller's cancel flag, seen by every workgroup after the barrier
    if (a.has_cancel && member == 0 && threadIdx.x == 0)
        stc(BATCH ? a.cword : &a.ctl->cancel, host_flag(a.cancel));
    if (!scope_barrier(y, BATCH ? a.bar : &a.ctl->barrier, members, epoch, &s_ok)) return;
    if (!BATCH && threadIdx.x == 0) {
        // every workgroup has counted itself into its XCD: the two-level
        // round barrier's member counts
        uint32_t n = 0;
        for (int i = 0; i < 16; ++i) n += ld_agent32(&a.ctl->xmem[i]) != 0u;
        s_xb.mx = ld_agent32(&a.ctl->xmem[s_xb.x]);
        s_xb.nx = n;
    }
    if constexpr (FFT) {
        if (!fft_spectrum<PT, Tile::kWide>(&a, y, &s_xb, &s_ok)) return;
    }

    const int64_t limit = a.max_iter < a.cap ? a.max_iter : a.cap;
    int64_t used = 0;
    int32_t rounds = 0, stop = STOP_MAXITER;
    double mflux = 0.0;
    uint64_t ph_local = 0, ph_gather = 0, ph_apply = 0, tp0 = 0, tp1 = 0;
    for (;;) {
        // ---- round control, computed identically by every workgroup: a tile
        // takes part when its peak is at or above the threshold and at or above
        // the round's flux level (level_frac times the largest tile peak); a
        // non-finite tile peak (magnitude bits at or above +Inf's) ends the run
        uint32_t vbits = 0;
        for (int t = threadIdx.x; t < T; t += WG) vbits = max(vbits, (uint32_t)(ldc(&a.tile_key[t]) >> 33));
        if (threadIdx.x == 0) s_vmax = 0;
        __syncthreads();
        if (vbits) atomicMax(&s_vmax, vbits);
        __syncthreads();
        const bool nonfinite = s_vmax >= 0x7F800000u;
        const bool cancelled = a.has_cancel && ldc(BATCH ? a.cword : &a.ctl->cancel) != 0u;
        const double level = nonfinite ? 0.0 : a.level_frac * (double)__uint_as_float(s_vmax);
        int na_part = 0, rk_part = 0;
        for (int t = threadIdx.x; t < T; t += WG) {
            const double pk = (double)fabsf(key_value(ldc(&a.tile_key[t])));
            const int act = pk >= a.threshold && pk >= level;
            na_part += act;
            rk_part += act && (t < tile);
        }
        const int na = wg_sum_int(na_part, &s_tmp);
        const int my_rank = wg_sum_int(rk_part, &s_tmp);
        if (used == a.max_iter) { stop = STOP_MAXITER; break; }
        if (cancelled) { stop = STOP_CANCELLED; break; }
        if (nonfinite) { stop = STOP_NONFINITE; break; }
        if (na == 0) { stop = STOP_THRESHOLD; break; }
        if (used == a.cap) { stop = STOP_CAPACITY; break; }
        const int64_t rem = limit - used;
        int64_t budget = 0;
        if (is_cluster) {
            const double pk = (double)fabsf(key_value(cur));
            const bool act = pk >= a.threshold && pk >= level;
            if (act) budget = rem >= (int64_t)na * a.interval ? a.interval
                                                                : rem / na + (my_rank < rem % na ? 1 : 0);
        }

        // ---- local minor loops
        if (member == 0) tp0 = wall_clock64();
        if (is_cluster) {
            int L = 0;
            bool aggregated = false;    // the round lists already written (multiplexed tiles)
            if constexpr (Tile::kWide) {
                // the cluster's tiles one after another (one tile unless the
                // clusters are time-multiplexed), each with its own key,
                // budget and round list
                const int ncl = BATCH ? T : a.ncl;
                for (int t = tile; t < T; t += ncl) {
                    uint64_t kt = cur;
                    int64_t bt = budget;
                    if (ncl < T) {
                        int ty0, tx0, th, tw;
                        tile_rect(a, t, ty0, tx0, th, tw);
                        R.init(im, ty0, tx0, th, tw, cs, rank, false);
                        kt = ldc(&a.tile_key[t]);
                        // this tile's budget: the round control's rule, with its
                        // rank among the active tiles
                        const double pk = (double)fabsf(key_value(kt));
                        const bool act = pk >= a.threshold && pk >= level;
                        int rk = 0;
                        for (int u = threadIdx.x; u < t; u += WG) {
                            const double pu = (double)fabsf(key_value(ldc(&a.tile_key[u])));
                            rk += pu >= a.threshold && pu >= level;
                        }
                        rk = wg_sum_int(rk, &s_tmp);
                        bt = !act ? 0
                                  : rem >= (int64_t)na * a.interval ? a.interval
                                                                     : rem / na + (rk < rem % na ? 1 : 0);
                    }
                    const WideRound wr =
                        (int64_t)R.h * R.w == (int64_t)R.stride() * WideTile<PT>::K
                            ? wide_round<PT, true>(a, im, R, y, slots, lslots, e, kt, bt, level, tile_leader_wg,
                                                   l_idx, l_flux)
                            : wide_round<PT, false>(a, im, R, y, slots, lslots, e, kt, bt, level, tile_leader_wg,
                                                    l_idx, l_flux);
                    if (!wr.ok) return;
                    e = wr.e;
                    if (ncl < T) {
                        if (tile_leader_wg) {
                            __syncthreads();
                            aggregate_round(a, t, wr.L, l_idx, l_flux, l_tmp, l_sum, &s_cnt);
                        }
                        __syncthreads();
                    } else {
                        cur = wr.cur;
                        L = wr.L;
                    }
                }
                aggregated = ncl < T;
                if (aggregated) {       // back to the first tile's geometry
                    int ty0, tx0, th, tw;
                    tile_rect(a, tile, ty0, tx0, th, tw);
                    R.init(im, ty0, tx0, th, tw, cs, rank, false);
                }
            } else
            for (int64_t it = 0; it < budget; ++it) {
                const float v = key_value(cur);
                if (!__builtin_isfinite(v) || (double)fabsf(v) < a.threshold || (double)fabsf(v) < level) break;
                const float c = a.gain * v;
                const uint32_t fp = key_f(cur);
                const int ly = (int)(fp / (uint32_t)R.w), lx = (int)(fp % (uint32_t)R.w);
                const int py = R.y0 + ly, px = R.x0 + lx;
                const int32_t img = py * a.nx + px;
                if (tile_leader_wg && threadIdx.x == 0) { l_idx[L] = img; l_flux[L] = c; }
                if (a.model && R.owns(fp)) a.model[img] += (double)c;
                const bool more = it + 1 < budget;
                const uint64_t tk = R.subtract(im, py, px, c, more);
                L += 1;
                if (more && !cluster_reduce(y, slots, lslots, a.slot_pad, cs, rank, e++, tk, cur)) return;
            }
            if (tile_leader_wg && !aggregated) {
                __syncthreads();
                aggregate_round(a, tile, L, l_idx, l_flux, l_tmp, l_sum, &s_cnt);
            }
        }
        if (!(BATCH ? scope_barrier(y, a.bar, members, epoch, &s_ok) : xcd_grid_barrier(y, &s_xb, &s_ok))) return;   // A
        if (member == 0) { tp1 = wall_clock64(); ph_local += tp1 - tp0; tp0 = tp1; }

        // ---- round bookkeeping: every workgroup reads the counts
        for (int t = threadIdx.x; t < T; t += WG) s_off[t + 1] = ldc(&a.rb_n[t]);
        __syncthreads();
        if (threadIdx.x == 0) {
            s_off[0] = 0;
            for (int t = 0; t < T; ++t) s_off[t + 1] += s_off[t];
        }
        __syncthreads();
        const int32_t nround = s_off[T];
        if (member == 0) {
            // append this round's components in (tile, local iteration) order
            double fsum = 0.0;
            for (int t = 0; t < T; ++t) {
                const int32_t cnt = s_off[t + 1] - s_off[t];
                for (int j = threadIdx.x; j < cnt; j += WG) {
                    const float fl = ldc(&a.rb_flux[(size_t)t * a.interval + j]);
                    a.comp_idx[used + s_off[t] + j] = ldc(&a.rb_idx[(size_t)t * a.interval + j]);
                    a.comp_flux[used + s_off[t] + j] = fl;
                    fsum += (double)fl;
                }
            }
            fsum = wave_sum64f(fsum);
            __shared__ double s_fs[NWAVES];
            if ((threadIdx.x & 63) == 0) s_fs[threadIdx.x >> 6] = fsum;
            __syncthreads();
            if (threadIdx.x == 0)
                for (int w = 0; w < NWAVES; ++w) mflux += s_fs[w];
        }
        used += nround;
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += WG) s_off[t + 1] = ldc(&a.ag_n[t]);
        __syncthreads();
        if (threadIdx.x == 0) {
            s_off[0] = 0;
            for (int t = 0; t < T; ++t) s_off[t + 1] += s_off[t];
        }
        __syncthreads();

        // ---- feedback by FFT: acc = component image (*) K, every tile's
        // components (apply then starts from the round's starting residual)
        if constexpr (FFT) {
            if constexpr (Tile::kWide) {
                if (!fft_feedback_wide<PT>(&a, y, &s_xb, &s_ok, s_off)) return;
            } else {
                if (!fft_feedback<PT, false>(a, y, &s_xb, &s_ok, s_off)) return;
            }
        } else
        // ---- feedback gather: acc[q] = sum over other tiles' components
        {
            // items are (tile, row band) in tile-major order; each XCD takes a
            // contiguous range of them so its L2 sees one compact PSF region
            // per component (workgroup b runs on XCD b % 8)
            const int parts = a.gather_parts;
            const int nitems = T * parts;
            const bool by_xcd = xcd_items && (members % 8) == 0;
            const int per_xcd_wg = by_xcd ? members / 8 : members;
            const int items_per_xcd = by_xcd ? (nitems + 7) / 8 : nitems;
            const int xcd = by_xcd ? member % 8 : 0;
            const int item_end = min(nitems, (xcd + 1) * items_per_xcd);
            for (int item = xcd * items_per_xcd + (by_xcd ? member / 8 : member);
                 item < item_end; item += per_xcd_wg) {
                const int s = item / parts, part = item % parts;
                int y0, x0, h, w;
                tile_rect(a, s, y0, x0, h, w);
                const int ngroups = (h * w) / V;
                const int per = (ngroups + parts - 1) / parts;
                const int g_lo = part * per;
                const int g_hi = min(ngroups, g_lo + per);
                const int32_t total = s_off[T] - (s_off[s + 1] - s_off[s]);
                for (int gb = g_lo; gb < g_hi; gb += WG * GATHER_M) {
                    float acc[GATHER_M][V];
                    int32_t goff[GATHER_M];
                    int64_t gimg[GATHER_M];
                    bool gv[GATHER_M];
#pragma unroll
                    for (int m = 0; m < GATHER_M; ++m) {
                        const int g = gb + m * WG + (int)threadIdx.x;
                        gv[m] = g < g_hi;
                        const int f = g * V;
                        const int y = f / w, x = f % w;
                        goff[m] = gv[m] ? (y0 + y) * a.psf_nx + (x0 + x) : 0;
                        gimg[m] = (int64_t)(y0 + y) * a.nx + (x0 + x);
#pragma unroll
                        for (int v = 0; v < V; ++v) acc[m][v] = 0.0f;
                    }
                    // components of tiles != s, in tile order, raster order inside a tile
                    for (int32_t c0 = 0; c0 < total; c0 += GATHER_CHUNK) {
                        const int32_t cn = min((int32_t)GATHER_CHUNK, total - c0);
                        __syncthreads();
                        for (int j = threadIdx.x; j < cn; j += WG) {
                            int32_t gi = c0 + j;                 // index in the list without tile s
                            if (gi >= s_off[s]) gi += s_off[s + 1] - s_off[s];
                            // find the tile of concatenated entry gi
                            int lo = 0, hi = T;                  // s_off[lo] <= gi < s_off[hi]
                            while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_off[mid] <= gi) lo = mid; else hi = mid; }
                            const size_t src = (size_t)lo * a.interval + (gi - s_off[lo]);
                            const int32_t pos = ldc(&a.ag_pos[src]);
                            const int py = pos / a.nx, px = pos % a.nx;
                            g_shift[j] = (a.cy - py) * a.psf_nx + (a.cx - px);
                            g_flux[j] = ldc(&a.ag_flux[src]);
                        }
                        __syncthreads();
                        // GATHER_J components at a time: all their PSF loads are
                        // issued before the fmas, which keep the component order
                        int j = 0;
                        for (; j + GATHER_J <= cn; j += GATHER_J) {
                            float fl[GATHER_J];
                            float pv[GATHER_J][GATHER_M][V];
#pragma unroll
                            for (int u = 0; u < GATHER_J; ++u) {
                                const int32_t sh = __builtin_amdgcn_readfirstlane(g_shift[j + u]);
                                fl[u] = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, g_flux[j + u])));
                                const char *base = (const char *)a.psf + (int64_t)sh * (int64_t)sizeof(PT);
                                const __amdgpu_buffer_rsrc_t rs =
                                    make_rsrc_uniform(base, a.psf_bytes - (uint64_t)sh * sizeof(PT));
#pragma unroll
                                for (int m = 0; m < GATHER_M; ++m)
                                    PsfLoad<PT, V>::load(rs, (uint32_t)goff[m] * (uint32_t)sizeof(PT), pv[u][m]);
                            }
#pragma unroll
                            for (int u = 0; u < GATHER_J; ++u)
#pragma unroll
                                for (int m = 0; m < GATHER_M; ++m)
#pragma unroll
                                    for (int v = 0; v < V; ++v) acc[m][v] = __builtin_fmaf(fl[u], pv[u][m][v], acc[m][v]);
                        }
                        for (; j < cn; ++j) {
                            const int32_t sh = __builtin_amdgcn_readfirstlane(g_shift[j]);
                            const float fl = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, g_flux[j])));
                            const char *base = (const char *)a.psf + (int64_t)sh * (int64_t)sizeof(PT);
                            const __amdgpu_buffer_rsrc_t rs =
                                make_rsrc_uniform(base, a.psf_bytes - (uint64_t)sh * sizeof(PT));
#pragma unroll
                            for (int m = 0; m < GATHER_M; ++m) {
                                float pv[V];
                                PsfLoad<PT, V>::load(rs, (uint32_t)goff[m] * (uint32_t)sizeof(PT), pv);
#pragma unroll
                                for (int v = 0; v < V; ++v) acc[m][v] = __builtin_fmaf(fl, pv[v], acc[m][v]);
                            }
                        }
                    }
#pragma unroll
                    for (int m = 0; m < GATHER_M; ++m)
                        if (gv[m]) {
#pragma unroll
                            for (int v = 0; v < V; ++v) stc(&a.accbuf[gimg[m] + v], acc[m][v]);
                        }
                }
            }
        }
        if (!(BATCH ? scope_barrier(y, a.bar, members, epoch, &s_ok) : xcd_grid_barrier(y, &s_xb, &s_ok))) return;   // B
        if (member == 0) { tp1 = wall_clock64(); ph_gather += tp1 - tp0; tp0 = tp1; }

        // ---- apply feedback and find each tile's new peak
        if (is_cluster) {
            if (!cluster_reduce(y, slots, lslots, a.slot_pad, cs, rank, e++, R.template apply_feedback<FFT>(im), cur)) return;
            if (tile_leader_wg && threadIdx.x == 0) stc(&a.tile_key[tile], cur);
            if constexpr (Tile::kWide && !BATCH) {
                // time-multiplexed clusters: the first tile above, then the others
                for (int t = tile + a.ncl; t < T; t += a.ncl) {
                    int ty0, tx0, th, tw;
                    tile_rect(a, t, ty0, tx0, th, tw);
                    R.init(im, ty0, tx0, th, tw, cs, rank, false);
                    uint64_t k;
                    if (!cluster_reduce(y, slots, lslots, a.slot_pad, cs, rank, e++, R.template apply_feedback<FFT>(im), k))
                        return;
                    if (tile_leader_wg && threadIdx.x == 0) stc(&a.tile_key[t], k);
                }
                if (a.ncl < T) {        // back to the first tile's geometry
                    int ty0, tx0, th, tw;
                    tile_rect(a, tile, ty0, tx0, th, tw);
                    R.init(im, ty0, tx0, th, tw, cs, rank, false);
                }
            }
        }
        rounds += 1;
        if (a.has_cancel && member == 0 && threadIdx.x == 0)
            stc(BATCH ? a.cword : &a.ctl->cancel, host_flag(a.cancel));
        if (!(BATCH ? scope_barrier(y, a.bar, members, epoch, &s_ok) : xcd_grid_barrier(y, &s_xb, &s_ok))) return;   // C
        if (member == 0) { tp1 = wall_clock64(); ph_apply += tp1 - tp0; }
    }

    // ---- results
    if (is_cluster) store_and_sum(R, im, a.partial, tile * cs + rank);
    if constexpr (Tile::kWide && !BATCH) {
        if (is_cluster) {
            for (int t = tile + a.ncl; t < T; t += a.ncl) {
                int ty0, tx0, th, tw;
                tile_rect(a, t, ty0, tx0, th, tw);
                R.init(im, ty0, tx0, th, tw, cs, rank, false);
                store_and_sum(R, im, a.partial, t * cs + rank);
            }
        }
    }
    if (member == 0 && threadIdx.x == 0) {
        uint64_t best = ldc(&a.tile_key[0]);
        for (int t = 1; t < T; ++t) {
            const uint64_t k = ldc(&a.tile_key[t]);
            if ((k >> 33) > (best >> 33)) best = k;       // largest |v|, lowest tile id on ties
        }
        a.dstat->n_iter = used;
        a.dstat->stop = stop;
        a.dstat->n_rounds = rounds;
        a.dstat->phase_ticks[0] = ph_local;
        a.dstat->phase_ticks[1] = ph_gather;
        a.dstat->phase_ticks[2] = ph_apply;
        a.dstat->final_peak = (double)key_value(best);
        a.dstat->model_flux = mflux;
    }
}

// Many independent images in one launch.  Problems are laid out largest
// first; problem i owns the seats [seat0[i], seat0[i+1]) and each seat is one
// workgroup of its cluster.
//
// Per-XCD schedule (when every XCD that holds workgroups holds at least the
// largest cluster's worth, counted at launch): each XCD pulls whole problems
// from the batch in order and runs them with its own workgroups, whose
// exchanges then stay in that XCD's L2.  Otherwise a workgroup takes the next
// seat of the whole batch from a device counter.  Either way tickets (seats)
// go out in order and every workgroup is resident, so the earliest
// unfinished problem always has all its members running: no deadlock.
template <class Tile, bool TILED> __global__ void __launch_bounds__(WG) batched_kernel(const BatchArgs b)
{
    __shared__ int s_work, s_ok;
    const Sync y{b.ctl, b.timeout_ticks};
    const int total = b.seat0[b.n];
    bool per_xcd = false;
    uint32_t x = 0;
    if (b.xcd_mode) {
        x = xcc_id();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&b.xq->count[x * XQ_STRIDE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t epoch = 0;
        if (!grid_barrier(y, epoch, &s_ok)) return;
        if (threadIdx.x == 0) {
            int ok = 1;
            for (int i = 0; i < XQ_N; ++i) {
                const uint32_t c = ld_agent32(&b.xq->count[i * XQ_STRIDE]);
                if (c != 0 && c < (uint32_t)b.max_cs) ok = 0;
            }
            s_work = ok;
        }
        __syncthreads();
        per_xcd = s_work != 0;
        __syncthreads();
    }
    for (;;) {
        // the next (problem << 12 | rank) for this workgroup, or -1
        if (threadIdx.x == 0) {
            int32_t w = -1;
            if (per_xcd) {
                w = xcd_ticket(b, y, x);
            } else {
                const int seat =
                    (int)__hip_atomic_fetch_add(&b.ctl->seat, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (seat < total) {
                    int lo = 0, hi = b.n;       // seat0[lo] <= seat < seat0[lo + 1]
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (b.seat0[mid] <= seat) lo = mid; else hi = mid;
                    }
                    w = (int32_t)(((uint32_t)lo << 12) | (uint32_t)(seat - b.seat0[lo]));
                }
            }
            s_work = w;
        }
        __syncthreads();
        const int32_t w = s_work;
        __syncthreads();
        if (w < 0) return;
        if constexpr (TILED) {
            const int ti = b.tiled_of[w >> 12];
            if (ti >= 0) {
                // member m of a tiled problem: tile m / cs, cluster rank m % cs
                const KArgs &ta = b.tjobs[ti];
                const int m = w & 0xFFF;
                tiled_body<Tile, false, true>(ta, m, b.jobs[w >> 12].cs, ((m / ta.cs) << 16) | (m % ta.cs), false);
                if (aborted(y)) return;
                continue;
            }
        }
        if (!run_plain<Tile>(b.jobs[w >> 12], w & 0xFFF, y, per_xcd, b.cancel, nullptr, 0)) return;
        if (aborted(y)) return;
    }
}


// Waves per SIMD the tiled kernel is compiled for: 4 (two 512-thread
// workgroups per CU, 128 registers) where the launches count on two
// co-resident workgroups per CU (the streamed tiles with the FFT feedback,
// and the 4-pixel register tiles with the direct feedback, whose clusters are
// the largest), else whatever the registers allow.
template <class Tile, bool FFT> __host__ __device__ constexpr int tiled_waves()
{
    if constexpr (Tile::kResident) return !FFT && Tile::kPx <= 4 ? 4 : 1;
    else return FFT && !Tile::kWide ? 4 : 1;
}

// The tiled form on the whole grid (one persistent, cooperative launch).
template <class Tile, bool FFT>
__global__ void __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(tiled_waves<Tile, FFT>())))
tiled_kernel(const KArgs a)
{
    // The argument block is used where it lies, in the kernel argument
    // segment (it is the only argument, at offset 0): the wide tiles pass its
    // address to their round functions, and a reference to the parameter
    // itself would make the compiler copy the block to every lane's private
    // memory first.
    (void)a;
    const KArgs &ka = *(const KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    tiled_body<Tile, FFT, false>(ka, 0, 0, ka.role[blockIdx.x], true);
}

// ------------------------------------------------------ small kernels ----

__global__ void finite_check_kernel(const float *x, int64_t n, uint32_t *flag)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= !__builtin_isfinite(x[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ void finite_check_half_kernel(const unsigned short *x, int64_t n, uint32_t *flag)
{
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad |= (x[i] & 0x7C00u) == 0x7C00u;
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

__global__ void to_half_kernel(const float *x, unsigned short *y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = __half_as_ushort(__float2half_rn(x[i]));
}

// y[i] = x[i + 1] (the last one 0): the FP16 PSF one element down, so that a
// window starting at an odd element starts on a 4-byte boundary in y.
__global__ void shift_half_kernel(const unsigned short *x, unsigned short *y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = i + 1 < n ? x[i + 1] : (unsigned short)0;
}

// Clear n 32-bit words (used where a fill must not be a runtime memset).
__global__ void zero_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Sum the per-workgroup squared-residual partials in a fixed order.
__global__ void finalize_kernel(const double *partial, int n, DevStat *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        st->sumsq = s;
    }
}

// The same for every problem of a batch (one thread per problem).
__global__ void finalize_batch_kernel(const PlainJob *jobs, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int r = 0; r < jobs[i].cs; ++r) s += jobs[i].partial[r];
    jobs[i].dstat->sumsq = s;
}

// ----------------------------------------------------- instantiations ----

#define INST(K, V, PT)                                                                   \
    template __global__ void hogbom_kernel<RegTile<K, V, PT>>(const KArgs a);           \
    template __global__ void batched_kernel<RegTile<K, V, PT>, false>(const BatchArgs b); \
    template __global__ void batched_kernel<RegTile<K, V, PT>, true>(const BatchArgs b);  \
    template __global__ void tiled_kernel<RegTile<K, V, PT>, false>(const KArgs a);     \
    template __global__ void tiled_kernel<RegTile<K, V, PT>, true>(const KArgs a);
#define INST_STREAM(V, PT)                                                               \
    template __global__ void hogbom_kernel<StreamTile<STREAM_K, V, PT>>(const KArgs a);  \
    template __global__ void tiled_kernel<StreamTile<STREAM_K, V, PT>, false>(const KArgs a); \
    template __global__ void tiled_kernel<StreamTile<STREAM_K, V, PT>, true>(const KArgs a);

template __global__ void tiled_kernel<WideTile<float>, false>(const KArgs a);
template __global__ void tiled_kernel<WideTile<float>, true>(const KArgs a);
template __global__ void tiled_kernel<WideTile<__half>, false>(const KArgs a);
template __global__ void tiled_kernel<WideTile<__half>, true>(const KArgs a);
#define INST_ALL_K(V, PT) INST(1, V, PT) INST(2, V, PT) INST(4, V, PT) INST(8, V, PT) INST(16, V, PT)
INST_ALL_K(4, float)
INST_ALL_K(4, __half)
INST(4, 1, float) INST(16, 1, float) INST(32, 1, float)
INST(4, 1, __half) INST(16, 1, __half) INST(32, 1, __half)
INST_STREAM(4, float) INST_STREAM(4, __half) INST_STREAM(1, float) INST_STREAM(1, __half)

} // namespace cleanhip
