// clean_device.h -- definitions shared by the gfx950 kernels and the host
// entry points of the CLEAN library (kernel arguments, device control block).
#pragma once
#include <stdint.h>

namespace cleanhip {

constexpr int WG = 512;                 // threads per workgroup (8 waves of 64)
constexpr int NWAVES = WG / 64;
constexpr int MAX_TILES = 1024;
constexpr int MAX_INTERVAL = 2048;
constexpr int GATHER_CHUNK = 2048;      // components staged in LDS per pass
constexpr int GATHER_M = 2;             // pixel groups per thread per gather pass
constexpr int GATHER_J = 8;             // components whose loads are issued together
constexpr int STREAM_K = 4;             // pixel groups per thread per streamed pass
constexpr int TWO_LEVEL_MIN_CS = 32;    // plain clusters this large exchange in two levels
constexpr int MAX_WG_PER_CU = 2;        // co-resident 512-thread workgroups the launches count on per CU
constexpr int FFT_MAX_LG = 13;          // one-level FFT transforms: length <= 8192 (64 KB of LDS)
constexpr int FFT_MAX_LG2 = 16;         // two-level FFT transforms: length <= 65536
constexpr int FFT_LDS_CPLX = 8960;       // LDS complex slots of the two-level passes (>= fft_pad_slots(8192))
                                         // (with the tiled kernel's static LDS, two workgroups fit one CU's 160 KB)
// LDS slots of a padded transform arena for a length-L axis (one spare slot
// after every 16 elements and one more after every 256), and the distance
// between the padded segments of a pass (odd).
__host__ __device__ constexpr int fft_pad_slots(int L) { return L + L / 16 + L / 256; }
__host__ __device__ constexpr int fft_seg_stride(int L) { return fft_pad_slots(L) | 1; }

enum { STOP_MAXITER = 0, STOP_THRESHOLD = 1, STOP_CAPACITY = 2, STOP_CANCELLED = 3, STOP_NONFINITE = 4 };
constexpr int64_t CANCEL_EVERY = 4096;  // plain: iterations between cancel checkpoints
constexpr double GATHER_MAX_BYTES = 17592186044416.0;   // 2^44: most PSF bytes one direct-gather round may read
enum : uint32_t { ABORT_TIMEOUT = 1u };

// Control words: each on its own 128-byte line.
struct DevCtl {
    uint32_t abort;
    uint32_t pad0[31];
    uint32_t barrier;
    uint32_t pad1[31];
    uint32_t finite_bad;
    uint32_t pad2[31];
    uint32_t seat;          // batched: next seat to hand out
    uint32_t pad3[31];
    uint32_t cancel;        // tiled: the caller's cancel flag as read before the last grid barrier
    uint32_t pad4[31];
    // tiled launches, the two-level round barrier: workgroups per XCD (counted
    // at launch), per-XCD arrival counters and release words (one line each),
    // and the counter the last arriver of each XCD arrives on
    uint32_t xmem[32];
    uint32_t xarr[16][32];
    uint32_t xrel[16][32];
    uint32_t xlead;
    uint32_t pad5[31];
};

struct DevStat {
    int64_t n_iter;
    int32_t stop;
    int32_t n_rounds;
    double final_peak;
    double model_flux;
    double sumsq;
    uint64_t phase_ticks[3];   // tiled: local loops, feedback gather, apply + re-peak (wall-clock ticks)
    int32_t xcd_local;         // clusters whose exchanges stayed inside one XCD
    int32_t levels;            // plain: 2 if the cluster exchanged in two levels, else 1 (0: not set)
};

// One plain CLEAN problem as a workgroup cluster sees it.
struct PlainJob {
    const float *dirty;
    float *residual;
    double *model;
    const void *psf;
    uint64_t psf_bytes;
    int ny, nx, psf_nx, cy, cx;
    int cs;                 // workgroups in the cluster
    int slot_pad;
    float gain;
    double threshold;
    int64_t max_iter;
    int64_t cap;
    int32_t *comp_idx;
    float *comp_flux;
    uint64_t *slots;        // [2][slot_pad] device-scope exchange slots
    uint64_t *lslots;       // [2][slot_pad] XCD-local exchange slots (batched), else null
    DevStat *dstat;
    double *partial;        // [cs]
};

// Per-XCD problem queues of the batched kernel (one 128-byte line per word),
// indexed by the 4-bit XCC id.
constexpr int XQ_STRIDE = 32;
constexpr int XQ_N = 16;
struct XcdQueue {
    uint32_t count[XQ_N * XQ_STRIDE];   // workgroups found on each XCD
    uint32_t next[XQ_N * XQ_STRIDE];    // next ticket of each XCD
    uint32_t front[XQ_N * XQ_STRIDE];   // tickets below this are assigned
    uint32_t closed[XQ_N * XQ_STRIDE];  // no problem left for this XCD
    uint32_t problem[XQ_STRIDE];        // next problem to hand out (all XCDs)
};

struct KArgs;

struct BatchArgs {
    const PlainJob *jobs;   // [n], largest first
    const int32_t *seat0;   // [n + 1] first seat of each problem
    int n;
    DevCtl *ctl;
    uint64_t timeout_ticks;
    int xcd_mode;           // try the per-XCD schedule (checked on the device)
    int max_cs;             // largest cluster of the batch
    int tickets;            // ticket slots per XCD (total seats)
    XcdQueue *xq;
    int32_t *xtable;        // [XQ_N][tickets] problem << 12 | rank per ticket
    const KArgs *tjobs;     // tiled problems' descriptions
    const int32_t *tiled_of;   // [n] index into tjobs of problem i, or -1 (plain)
    const int32_t *cancel;  // the caller's cancel flag (host memory), or null
};

struct KArgs {
    const float *dirty;
    float *residual;
    double *model;
    const void *psf;
    const void *psf1;       // FP16 PSF moved down one element (psf1[i] = psf[i + 1]) for the wide tile's
                            // odd-element windows, which then start on a 4-byte boundary; or null
    uint64_t psf_bytes;
    int ny, nx, psf_ny, psf_nx, cy, cx;
    int ty, tx, T;
    int cs;                 // workgroups per tile cluster
    int ncl;                // tile clusters; below T (wide tile only) a cluster runs
                            // tiles c, c + ncl, ... one after another in each round
    int slot_pad;           // u64 slots per parity block of a cluster
    int interval;           // feedback interval (tiled)
    double level_frac;      // flux trigger: fraction of the largest tile peak (0: off)
    int gather_parts;       // gather work items per tile
    float gain;
    double threshold;
    int64_t max_iter;
    int64_t cap;
    uint64_t timeout_ticks;
    int32_t *comp_idx;
    float *comp_flux;
    const int32_t *cancel;  // the caller's cancel flag (host memory), or null
    int has_cancel;         // cancel != null
    // workspace
    DevCtl *ctl;
    uint32_t *bar;          // the rounds' barrier counter: &ctl->barrier, or a batched problem's own
    uint32_t *cword;        // the cancel flag as read before a barrier: &ctl->cancel, or the problem's own
    DevStat *dstat;
    const int32_t *role;    // per workgroup: tile << 16 | rank, or -1 (helper)
    uint64_t *xslots;       // [T][2][slot_pad] device-scope exchange slots
    uint64_t *lslots;       // [T][2][slot_pad] XCD-local exchange slots
    uint64_t *hslots;       // plain, cs >= TWO_LEVEL_MIN_CS: [2][8 * hpad + 32] two-level slots, else null
    int hpad;
    uint64_t *tile_key;     // [T]
    int32_t *rb_idx;        // [T][interval] raw round lists
    float *rb_flux;
    int32_t *rb_n;          // [T]
    int32_t *ag_pos;        // [T][interval] aggregated round lists (ascending position)
    float *ag_flux;
    int32_t *ag_n;          // [T]
    float *accbuf;          // [ny*nx] feedback sums
    // FFT form of the feedback (fft_lgx = 0: direct gather)
    int fft_lgx, fft_lgy;   // log2 of the transform sizes Lx, Ly (0: direct gather)
    int fft_two_x, fft_two_y;  // axis uses two-level transforms
    float2 *fft_b;          // [Lx/2+1][max(ny, Ly)] carried x bins of every row, by column
    float2 *fft_wx;         // [max(ny, Ly)/2][Lx] two-level x work rows (row pairs)
    float2 *fft_wy;         // [Lx/2+1][Ly] two-level y work columns
    float2 *fft_ks;         // [Lx/2+1][Ly] spectrum of the PSF kernel by carried column
    float *comp_img;        // [ny*nx] dense component image (two-level x), zero between rounds
    const float2 *tw_x;     // [Lx] twiddles exp(-2 pi i m / Lx)
    const float2 *tw_y;     // [Ly]
    float *rstart;          // [ny*nx] residual at the round's start (FFT form), else null
    double *partial;        // [T*cs] per-workgroup sum of squared residuals
};

} // namespace cleanhip
