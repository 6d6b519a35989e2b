/* Drives the oracle (test infrastructure, never part of the product path)
 * over every kind, symbol width and edge case so that a build of the oracle
 * with AddressSanitizer and UndefinedBehaviorSanitizer can report any
 * out-of-bounds access, leak or undefined operation.  Exits non-zero when a
 * call returns a code other than the expected one. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_build(int kind, const void* S, int sym_bytes, uint64_t n, uint32_t sigma, int arity_log2,
                 const uint64_t* codes, const uint32_t* lens, uint8_t** image, uint64_t* image_bytes);
int oracle_huffman(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* lens);
void oracle_free(void* p);

enum { K_WT = 1, K_WM = 2, K_SHAPED = 3, K_MULTI = 4 };

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void)   /* xorshift64 */
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
}

static int failures = 0;

static void expect(int got, int want, const char* what, int kind, uint64_t n, uint32_t sigma, int w)
{
    if (got != want) {
        fprintf(stderr, "%s kind=%d n=%llu sigma=%u width=%d: got %d, want %d\n", what, kind,
                (unsigned long long)n, sigma, w, got, want);
        failures++;
    }
}

/* n symbols below sigma (skewed: small values frequent), stored w bytes wide */
static void* make_sequence(uint64_t n, uint32_t sigma, int w, uint32_t absent)
{
    void* S = malloc(n ? n * (uint64_t)w : 1);
    for (uint64_t i = 0; i < n; i++) {
        uint32_t x = (uint32_t)(next_u64() % sigma);
        if (next_u64() & 1) x = (uint32_t)(x % (sigma < 7 ? sigma : 7));
        if (sigma > 1 && x == absent) x = (absent + 1) % sigma;   /* one symbol never occurs */
        if (w == 1) ((uint8_t*)S)[i] = (uint8_t)x;
        else if (w == 2) ((uint16_t*)S)[i] = (uint16_t)x;
        else ((uint32_t*)S)[i] = x;
    }
    return S;
}

static void build_all_kinds(const void* S, uint64_t n, uint32_t sigma, int w)
{
    uint8_t* img;
    uint64_t bytes;
    expect(oracle_build(K_WT, S, w, n, sigma, 1, NULL, NULL, &img, &bytes), 0, "tree", K_WT, n, sigma, w);
    oracle_free(img);
    expect(oracle_build(K_WM, S, w, n, sigma, 1, NULL, NULL, &img, &bytes), 0, "matrix", K_WM, n, sigma, w);
    oracle_free(img);
    for (int D = 1; D <= 4; D++) {
        expect(oracle_build(K_MULTI, S, w, n, sigma, D, NULL, NULL, &img, &bytes), 0, "multiary", K_MULTI, n,
               sigma, w);
        oracle_free(img);
    }
    /* shaped by the canonical Huffman code of the counts (absent symbols get
       no codeword), then by a code that also gives absent symbols codewords */
    uint64_t* counts = calloc(sigma, sizeof(uint64_t));
    uint64_t* codes = calloc(sigma, sizeof(uint64_t));
    uint32_t* lens = calloc(sigma, sizeof(uint32_t));
    for (uint64_t i = 0; i < n; i++) {
        const uint32_t x = w == 1 ? ((const uint8_t*)S)[i] : w == 2 ? ((const uint16_t*)S)[i] : ((const uint32_t*)S)[i];
        counts[x]++;
    }
    if (oracle_huffman(counts, sigma, codes, lens) == 0) {
        /* an empty sequence gives no codeword at all: no tree to shape */
        expect(oracle_build(K_SHAPED, S, w, n, sigma, 1, codes, lens, &img, &bytes), n ? 0 : -1, "shaped",
               K_SHAPED, n, sigma, w);
        oracle_free(img);
    }
    for (uint32_t x = 0; x < sigma; x++) counts[x] += 1;
    if (sigma <= 4096 && oracle_huffman(counts, sigma, codes, lens) == 0) {
        expect(oracle_build(K_SHAPED, S, w, n, sigma, 1, codes, lens, &img, &bytes), 0, "shaped, full code",
               K_SHAPED, n, sigma, w);
        oracle_free(img);
    }
    free(counts);
    free(codes);
    free(lens);
}

int main(void)
{
    static const uint64_t ns[] = {0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 20000, 70001};
    static const uint32_t sigmas[] = {1, 2, 3, 5, 64, 255, 256, 1000, 65536, 70000};
    for (size_t a = 0; a < sizeof ns / sizeof ns[0]; a++)
        for (size_t b = 0; b < sizeof sigmas / sizeof sigmas[0]; b++)
            for (int w = 1; w <= 4; w *= 2) {
                const uint32_t sigma = sigmas[b];
                if ((w == 1 && sigma > 256) || (w == 2 && sigma > 65536)) continue;
                if (sigma > 1000 && ns[a] != 0 && ns[a] != 1 && ns[a] != 4097) continue;   /* keep the run short */
                void* S = make_sequence(ns[a], sigma, w, sigma / 2);
                build_all_kinds(S, ns[a], sigma, w);
                free(S);
            }
    /* a symbol >= sigma is refused */
    {
        uint16_t S[5] = {0, 1, 2, 9, 1};
        uint8_t* img;
        uint64_t bytes;
        expect(oracle_build(K_WM, S, 2, 5, 4, 1, NULL, NULL, &img, &bytes), -2, "out of range", K_WM, 5, 4, 2);
        oracle_free(img);
    }
    /* Huffman over random counts with zeros, and a skew that needs long codes */
    for (int r = 0; r < 50; r++) {
        const uint32_t sigma = 1 + (uint32_t)(next_u64() % 3000);
        uint64_t* counts = calloc(sigma, sizeof(uint64_t));
        uint64_t* codes = calloc(sigma, sizeof(uint64_t));
        uint32_t* lens = calloc(sigma, sizeof(uint32_t));
        for (uint32_t x = 0; x < sigma; x++) counts[x] = (next_u64() % 4) ? next_u64() % 1000 : 0;
        if (r % 10 == 9)
            for (uint32_t x = 0; x < sigma && x < 60; x++) counts[x] = 1ull << (x < 50 ? x : 50);
        const int rc = oracle_huffman(counts, sigma, codes, lens);
        if (rc != 0 && rc != -5) expect(rc, 0, "huffman", 0, 0, sigma, 0);
        free(counts);
        free(codes);
        free(lens);
    }
    if (failures) fprintf(stderr, "%d failures\n", failures);
    else printf("oracle driver: all calls returned the expected codes\n");
    return failures ? 1 : 0;
}
