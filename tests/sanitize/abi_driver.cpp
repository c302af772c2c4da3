// Host-side checks of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (linked with a host-sanitized clean_api object,
// no GPU needed): every entry point's argument validation, the workspace
// size arithmetic over a sweep of shapes, and the status strings.  Fake
// device pointers are never dereferenced on these paths.  Exit status 0 when
// every call returns what the header documents.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "clean.h"

static int failures = 0;
#define EXPECT(cond)                                                            \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);      \
            ++failures;                                                         \
        }                                                                       \
    } while (0)

int main()
{
    void *F = reinterpret_cast<void *>(0x1000);
    float *ff = static_cast<float *>(F);
    int32_t *fi = static_cast<int32_t *>(F);
    clean_params p;
    std::memset(&p, 0, sizeof p);
    p.gain = 0.1;
    p.max_iter = 100;

    for (int s = -8; s <= 2; ++s) EXPECT(clean_strerror(s) != nullptr && clean_strerror(s)[0] != 0);
    EXPECT(std::strstr(clean_version(), "gfx950") != nullptr);

    // plain and tiled argument errors: nothing is touched
    EXPECT(clean_hogbom(nullptr, 16, 16, F, 32, 32, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_hogbom(ff, 16, 16, F, 31, 32, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_hogbom(ff, 0, 16, F, 32, 32, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_hogbom(ff, 16, 16, F, 32, 32, nullptr, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_last_error()[0] != 0);
    clean_params bad = p;
    bad.gain = -1.0;
    EXPECT(clean_hogbom(ff, 16, 16, F, 32, 32, &bad, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    bad = p;
    bad.px_per_thread = -4;
    EXPECT(clean_hogbom(ff, 16, 16, F, 32, 32, &bad, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    bad = p;
    bad.threshold = -1.0;
    EXPECT(clean_hogbom(ff, 16, 16, F, 32, 32, &bad, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_hogbom(ff, 16384, 32768, F, 32768, 65536, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr,
                        nullptr) == CLEAN_E_UNSUPPORTED);   // 2^29 pixels
    EXPECT(clean_hogbom_noalloc(nullptr, 16, 16, F, 32, 32, &p, ff, fi, ff, 100, nullptr, nullptr, nullptr) ==
           CLEAN_E_INVAL);
    EXPECT(clean_tiled_feedback(ff, 16, 16, F, 32, 32, 0, 2, 10, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr,
                                nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_tiled_feedback(ff, 16, 16, F, 32, 32, 2, 2, 0, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr,
                                nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_tiled_feedback(ff, 16, 16, F, 32, 32, 20, 2, 10, &p, ff, fi, ff, 100, nullptr, nullptr, 0, nullptr,
                                nullptr) == CLEAN_E_INVAL);

    // batched: problem validation, sizes of the batch
    clean_stats st[2];
    std::vector<clean_problem> probs(2);
    std::memset(probs.data(), 0, sizeof(clean_problem) * probs.size());
    EXPECT(clean_batched(nullptr, 1, &p, st, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_batched(probs.data(), -1, &p, st, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_batched(probs.data(), 70000, &p, st, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_batched(probs.data(), 0, &p, st, nullptr) == CLEAN_OK);
    for (auto &q : probs) {
        q.dirty = ff; q.psf = F; q.residual = ff; q.comp_idx = fi; q.comp_flux = ff;
        q.comp_cap = 10; q.max_iter = 10; q.ny = 16; q.nx = 16; q.psf_ny = 16; q.psf_nx = 32;
    }
    EXPECT(clean_batched(probs.data(), 2, &p, st, nullptr) == CLEAN_E_INVAL);
    EXPECT(std::strstr(clean_last_error(), "problem 0") != nullptr);
    int ppt = 7;
    float ms[CLEAN_BATCH_TUNE_CANDIDATES];
    EXPECT(clean_autotune_batched(probs.data(), 2, &p, 100, &ppt, ms, nullptr) == CLEAN_E_INVAL);
    EXPECT(ppt == 0);
    EXPECT(clean_autotune_batched(probs.data(), 2, &p, 0, &ppt, ms, nullptr) == CLEAN_E_INVAL);

    // tuners
    clean_params best;
    EXPECT(clean_autotune(ff, 16, 16, F, 32, 32, 1, 1, 1, &p, ff, fi, ff, 100, 0, &best, nullptr) == CLEAN_E_INVAL);
    const int grids[4] = {2, 2, 4, 4}, ivs[2] = {10, 50};
    clean_plan plan;
    EXPECT(clean_autotune_plan(ff, 16, 16, F, 32, 32, grids, 2, ivs, 2, &p, 100, 0.05, 0.1, nullptr, &plan,
                               nullptr, nullptr, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_autotune_plan(ff, 16, 16, F, 32, 32, nullptr, 2, ivs, 2, &p, 100, -0.1, 0.1, nullptr, &plan,
                               nullptr, nullptr, nullptr) == CLEAN_E_INVAL);

    // restoration and conversion
    int64_t area = 0;
    double sigma = 0.0;
    EXPECT(clean_beam_fit(nullptr, 32, 32, CLEAN_PSF_F32, &area, &sigma, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_restore(nullptr, ff, 16, 16, 2.0, nullptr, nullptr) == CLEAN_E_INVAL);
    EXPECT(clean_psf_to_f16(nullptr, nullptr, 10, nullptr) == CLEAN_E_INVAL);
    double gbs = 0.0;
    EXPECT(clean_bandwidth_probe(nullptr, 1 << 20, 0, 1, &gbs, nullptr) == CLEAN_E_INVAL);

    // workspace sizes: a sweep of shapes, tile grids, intervals and flags
    // (the size arithmetic in 64 bits, no overflow), and the limit's get/set
    const int sides[] = {1, 2, 7, 64, 255, 1024, 4097, 16384, 32768};
    size_t sum = 0;
    for (int ny : sides)
        for (int nx : sides)
            for (int t : {1, 2, 3, 16})
                for (int ivl : {1, 100, 2048})
                    for (int flags : {0, (int)CLEAN_FLAG_FFT_FEEDBACK, (int)(CLEAN_FLAG_FFT_FEEDBACK | CLEAN_FLAG_FFT_TWO_LEVEL)}) {
                        clean_params q = p;
                        q.flags = flags;
                        sum += clean_workspace_size(ny, nx, t, t, ivl, &q);
                    }
    EXPECT(sum > 0);
    EXPECT(clean_workspace_size(0, 16, 1, 1, 1, &p) == 0);
    EXPECT(clean_workspace_size(16, 16, 1, 1, 1, nullptr) == 0);
    const size_t old = clean_set_workspace_limit(123456789);
    EXPECT(clean_set_workspace_limit(old) == 123456789);

    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("abi driver: all checks passed\n");
    return 0;
}
