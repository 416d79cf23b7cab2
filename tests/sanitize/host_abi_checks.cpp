// Host sanitizer run of the library's host side (tests/test_sanitizers_host.py
// builds the library's sources with address and undefined-behaviour
// sanitizers on the host pass only): sizing, binding, the build planners of
// one text, a pair, a batch, the conversion, the merge, the sorting build and
// the position map, and every argument error path, over many sizes.  Nothing
// here reaches the device: every call returns before it would enqueue work
// (fake device pointers are never dereferenced on the host).
#include <cstdint>
#include <cstdio>
#include <vector>

#include "wt.h"

static int failures = 0;
#define CHECK(c, msg)                                      \
    do {                                                   \
        if (!(c)) {                                        \
            std::fprintf(stderr, "check failed: %s\n", msg); \
            failures++;                                    \
        }                                                  \
    } while (0)

int main()
{
    const uint64_t sizes[] = {0, 1, 63, 64, 65, 4097, 1u << 20, (1u << 26) + 3, 3000000000ull};
    void *fake = (void *)(uintptr_t)(1ull << 40);
    for (uint64_t n : sizes)
        for (uint32_t L = 0; L <= 32; L += (L < 9 ? 1 : 5)) {
            const size_t out = wt_output_bytes(n, L);
            CHECK(out > 0, "output bytes");
            for (uint32_t b : {1u, 2u, 4u}) {
                for (int kind = 0; kind < 2; kind++) {
                    wt_tune tune = {0, 3, 7, 11};
                    (void)wt_workspace_bytes(n, b, L, (wt_kind)kind);
                    (void)wt_workspace_bytes_tuned(n, b, L, (wt_kind)kind, &tune);
                }
                (void)wt_pair_workspace_bytes(n, b, L);
                (void)wt_ps_workspace_bytes(n, b, L);
            }
            (void)wt_convert_workspace_bytes(n, L);
            (void)wt_merge_workspace_bytes(n, L, 7);
            (void)wt_export_pool_words(n, L);
            (void)wt_posmap_bytes(n, L);
            for (int kind = 0; kind < 2; kind++) {
                wt_levels v;
                CHECK(wt_levels_bind(&v, fake, out, n, L, (wt_kind)kind) == WT_OK, "bind");
                // wt_output_bytes holds 256 bytes of alignment slack
                CHECK(wt_levels_bind(&v, fake, out - 257, n, L, (wt_kind)kind) == WT_ENOSPACE, "bind too small");
                // argument errors return before any device work
                CHECK(wt_build_tuned((wt_kind)kind, fake, n, 3, L, &v, fake, 1 << 30, nullptr, nullptr) == WT_EINVAL,
                      "bad width");
                CHECK(wt_build_tuned((wt_kind)kind, fake, n, 1, L, &v, nullptr, 1 << 30, nullptr, nullptr) != WT_OK,
                      "no workspace");
                CHECK(wt_build_tuned((wt_kind)kind, fake, n, 1, L, &v, fake, 16, nullptr, nullptr) != WT_OK || L == 0,
                      "workspace too small");
                CHECK(wt_pair_build(fake, n, 3, L, &v, &v, fake, 1 << 30, nullptr) == WT_EINVAL, "pair bad width");
                CHECK(wt_pair_build_noalloc(fake, n, 3, L, &v, &v, nullptr) == WT_EINVAL, "noalloc bad width");
                CHECK(wt_access(&v, nullptr, 5, nullptr, nullptr) == WT_EINVAL, "access nulls");
            }
        }
    // batch planning over mixed items, with tunes
    std::vector<wt_levels> views(64);
    std::vector<wt_batch_item> items(64);
    for (uint32_t i = 0; i < 64; i++) {
        const uint64_t n = (i * 7919u) % 5000u;
        const uint32_t L = (i % 3 == 0) ? 2u : ((i % 3 == 1) ? 8u : 16u);
        const uint32_t b = L <= 8 ? 1u : 2u;
        wt_levels_bind(&views[i], fake, wt_output_bytes(n, L), n, L, (wt_kind)(i % 2));
        items[i] = wt_batch_item{fake, n, b, L, i % 2, 0, &views[i]};
    }
    for (uint32_t g : {0u, 1u, 3u, 128u})
        for (uint32_t p : {0u, 17u, 4096u}) {
            wt_tune tune = {0, 0, g, p};
            const size_t ws = wt_batch_workspace_bytes(items.data(), 64, &tune);
            CHECK(ws > 0, "batch workspace");
            CHECK(wt_batch_build(items.data(), 64, fake, 16, &tune, nullptr) == WT_ENOSPACE, "batch too small");
        }
    CHECK(wt_batch_build(nullptr, 3, fake, 1 << 20, nullptr, nullptr) == WT_EINVAL, "batch nulls");
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host sanitizer checks ok\n");
    return 0;
}
