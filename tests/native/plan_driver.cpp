// Drives the host side of the library (planning of every kind, node tables
// of shaped trees, batch planning, canonical Huffman codes, argument checks)
// so that a host build with AddressSanitizer and UndefinedBehaviorSanitizer
// can report any out-of-bounds access, leak or undefined operation.  No call
// here touches a GPU.  Exits non-zero when a call returns a code outside the
// set it may return.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "wavelet.h"

namespace {

uint64_t state = 0x2545F4914F6CDD1Dull;
uint64_t next_u64()   // xorshift64
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

int failures = 0;

void allow(int rc, std::initializer_list<int> ok, const char* what)
{
    for (int c : ok)
        if (rc == c) return;
    std::fprintf(stderr, "%s: unexpected code %d (%s)\n", what, rc, wt_strerror(rc));
    failures++;
}

void plans()
{
    const uint64_t ns[] = {0, 1, 63, 64, 8191, 8192, 8193, 100000, 1ull << 24, (1ull << 32) - 1, 1ull << 32};
    const uint32_t sigmas[] = {1, 2, 3, 200, 256, 257, 65536, 65537, 1u << 20, 0xFFFFFFFFu};
    const uint32_t widths[] = {1, 2, 4, 3};
    for (uint64_t n : ns)
        for (uint32_t sigma : sigmas)
            for (uint32_t w : widths)
                for (int kind : {WT_KIND_WT, WT_KIND_WM, WT_KIND_MULTIARY, 7})
                    for (uint32_t tau : {0u, 1u, 5u, 8u, 9u})
                        for (uint32_t tile : {0u, 1u, 16u}) {
                            wt_tuning t{tau, tile, 0, tau == 1 ? (uint32_t)WT_FLAG_LEVELWISE : 0u};
                            wt_shape sh{};
                            sh.arity_log2 = kind == WT_KIND_MULTIARY ? 1 + (uint32_t)(next_u64() % 4) : 0;
                            wt_plan_info info;
                            const int rc = wt_plan(kind, n, sigma, w, kind == WT_KIND_MULTIARY ? &sh : nullptr,
                                                   &t, &info);
                            allow(rc, {WT_OK, WT_EINVAL, WT_EUNSUP}, "wt_plan");
                        }
}

void shaped_plans()
{
    for (int r = 0; r < 200; r++) {
        const uint32_t sigma = 1 + (uint32_t)(next_u64() % (r < 150 ? 300 : 70000));
        std::vector<uint64_t> counts(sigma), codes(sigma);
        std::vector<uint32_t> lens(sigma);
        for (auto& c : counts) c = (next_u64() % 3) ? next_u64() % 5000 : 0;
        if (r % 17 == 0)
            for (uint32_t x = 0; x < sigma && x < 60; x++) counts[x] = 1ull << (x < 50 ? x : 50);
        const int hc = wt_huffman_codes(counts.data(), sigma, codes.data(), lens.data());
        allow(hc, {WT_OK, WT_EUNSUP}, "wt_huffman_codes");
        if (hc != WT_OK) continue;
        uint64_t n = 0;
        for (auto c : counts) n += c;
        // damage the code now and then: a codeword that is a prefix of
        // another, a length past 32, a codeword wider than its length
        if (r % 5 == 1 && sigma > 2) lens[1] = lens[1] ? lens[1] + 40 : 0;
        if (r % 5 == 2 && sigma > 2 && lens[0] > 1) lens[0] -= 1;
        if (r % 5 == 3 && sigma > 2) codes[2] |= 1ull << 40;
        wt_shape sh{0, 0, codes.data(), lens.data(), counts.data()};
        wt_plan_info info;
        allow(wt_plan(WT_KIND_SHAPED, n, sigma, 4, &sh, nullptr, &info), {WT_OK, WT_EINVAL, WT_EUNSUP},
              "wt_plan shaped");
    }
}

void batch_plans()
{
    for (int r = 0; r < 40; r++) {
        const uint32_t count = 1 + (uint32_t)(next_u64() % 300);
        std::vector<wt_seq_desc> ds(count);
        for (auto& d : ds) {
            d.S = (const void*)(uintptr_t)4096;
            d.n = next_u64() % (r % 4 == 0 ? (1ull << 24) : 100000);
            d.sigma = 1 + (uint32_t)(next_u64() % (1u << 20));
            d.sym_bytes = 4;
            d.out = (void*)(uintptr_t)8192;
            d.out_bytes = 1ull << 40;
            d.tau = (uint32_t)(next_u64() % 9);
            d.reserved = 0;
        }
        if (r % 7 == 3) ds[0].sym_bytes = 3;
        if (r % 7 == 4) ds[count - 1].out_bytes = 8;
        wt_tuning t{0, (uint32_t)(next_u64() % 20), 0, 0};
        uint64_t ws = 0;
        allow(wt_batch_plan(WT_KIND_WM, ds.data(), count, r % 2 ? &t : nullptr, &ws),
              {WT_OK, WT_EINVAL, WT_ENOSPC, WT_EUNSUP}, "wt_batch_plan");
    }
    uint64_t ws = 0;
    allow(wt_batch_plan(WT_KIND_WM, nullptr, 0, nullptr, &ws), {WT_OK, WT_EINVAL}, "empty batch");
    allow(wt_batch_plan(WT_KIND_WT, nullptr, 0, nullptr, &ws), {WT_EINVAL}, "batch of trees");
}

}  // namespace

int main()
{
    plans();
    shaped_plans();
    batch_plans();
    for (int c = -10; c <= 1; c++) (void)wt_strerror(c);
    if (failures) std::fprintf(stderr, "%d failures\n", failures);
    else std::printf("plan driver: every call returned an allowed code\n");
    return failures ? 1 : 0;
}
