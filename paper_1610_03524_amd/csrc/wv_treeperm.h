// wv_treeperm.h -- tree levels gathered from wavelet-matrix levels.
#pragma once

#include <vector>

#include "wv_internal.h"

// one kept run of a level: `len` bits from bit `src` of the matrix level go
// to bit `dst` of the tree level (runs of a level ordered by dst, covering it)
struct wv_perm_seg {
    uint64_t dst, src, len;
};

// one tree level to gather
struct wv_perm_level {
    uint64_t* dst;          // tree level words (in the image)
    const uint64_t* src;    // matrix level words (one readable word past the end)
    uint64_t nbits;         // bits on the tree level
    uint64_t seg0, nseg;    // its runs in the segment array
    uint16_t* sub;          // multiary: the level's sub-range counters (counting launch only)
};

// Counters of multiary levels taken while gathering them (levels of D-bit
// digits; m = the digits of every level in the gather of balanced trees from
// symbol groups, the gather of runs takes each level's own length).
// rng_cnt[(r * M + l) * 2^D + g] receives the number of digits g in 64-word
// range r of level l (rows past a shorter level's ranges are not written),
// and each level's sub-range counters are written.
struct wv_perm_counts {
    uint32_t* rng_cnt;
    uint64_t m;
    uint32_t D, M;
};

// output words per workgroup of the gather (one per thread)
constexpr uint32_t WV_PERM_TILE = 256;

// The gather's tiles: level l covers tiles tile0[l] .. tile0[l+1]-1 (its
// words, or with `counting` its whole 64-word counter ranges, in tiles of
// WV_PERM_TILE words), and tile_seg[t] is the run holding the first bit of
// tile t (the last run of its level when the tile starts past the level's
// bits).  Returns the number of tiles.
uint32_t wv_tree_tiles(const std::vector<wv_perm_level>& lv, const std::vector<wv_perm_seg>& segs, bool counting,
                       std::vector<uint32_t>& tile0, std::vector<uint32_t>& tile_seg);

// upper bound of the tiles of nlev levels of at most n symbols of D bits
inline uint64_t wv_tree_tile_bound(uint64_t n, uint32_t D, uint32_t nlev)
{
    const uint64_t words = wv_cdiv(wv_cdiv(n * D, 64), 64) * 64;
    return (uint64_t)nlev * (wv_cdiv(words, WV_PERM_TILE) + 1) + 1;
}

// Runs of every level 0..key_bits-1 from the symbol counts.  Balanced tree:
// codes == nullptr, key = symbol.  Shaped tree: key = codes[x] padded at the
// bottom to key_bits (the longest code length), symbols whose code is no
// longer than l are left out of level l.  seg0[l] = first run of level l,
// seg0[key_bits] = number of runs.
void wv_tree_segments(const std::vector<uint64_t>& counts, uint32_t key_bits, const uint32_t* codes,
                      const uint32_t* lens, std::vector<wv_perm_seg>& segs, std::vector<uint64_t>& seg0);

// keys[i] = ktab[S[i]] (device table; 0 for S[i] >= sigma)
hipError_t wv_tree_keys(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma, const uint32_t* ktab,
                        uint32_t* keys, hipStream_t s);
// the padded-key table: codes[x] << (h - lens[x]) for every coded symbol, else 0
void wv_key_table(const uint32_t* codes, const uint32_t* lens, uint32_t sigma, uint32_t h, std::vector<uint32_t>& tab);

// Shaped trees with codes longer than WV_SPLIT_BITS whose symbols make at most
// 1/WV_SPLIT_SHARE of the sequence are built from two matrices: one over the
// top WV_SPLIT_BITS bits of every padded codeword (levels above the split),
// one over the whole codewords of the long-code symbols alone, in input order
// (the levels below it, where only those symbols remain).
constexpr uint32_t WV_SPLIT_BITS = 16;
constexpr uint64_t WV_SPLIT_SHARE = 8;

// blocks of the two key kernels below
uint64_t wv_tree_key_blocks(uint64_t n);

// the split table of every symbol x < sigma: the top h1 bits of its code
// padded to h bits, plus WV_SPLIT_LONG when the code is longer than h1 (0 for
// symbols without a code)
constexpr uint32_t WV_SPLIT_LONG = 1u << 16;
void wv_split_table(const uint32_t* codes, const uint32_t* lens, uint32_t sigma, uint32_t h, uint32_t h1,
                    std::vector<uint32_t>& tab);

// keys[i] = the low 16 bits of ktab[S[i]] (0 for S[i] >= sigma); bcnt[b] =
// symbols of block b whose code is longer than h1
hipError_t wv_tree_keys_split(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma, const uint32_t* ktab,
                              uint16_t* keys, uint32_t* bcnt, uint16_t* lmask, hipStream_t s);
// bytes of the long-code marks the split key kernel leaves for the long keys
uint64_t wv_tree_lmask_bytes(uint64_t n, uint32_t sym_bytes);

// lkeys[r] = padded codeword (codes[x] << (h - lens[x])) of the r-th symbol,
// in input order, whose code is longer than h1, found from the marks the
// split key kernel left in lmask (S is read only at marked positions); boff
// = exclusive prefix of bcnt.  Ranks >= nlong are not written (a sequence
// whose counts differ from the shape is rejected later).
hipError_t wv_tree_long_keys(const void* S, uint64_t n, uint32_t sym_bytes, const uint32_t* codes, const uint32_t* lens,
                             uint32_t h, const uint64_t* boff, const uint16_t* lmask, uint32_t* lkeys, uint64_t nlong,
                             hipStream_t s);

// matrix levels bD .. bD+D-1 (words and rank directories) of one multiary level
struct wv_digit_levels {
    const uint64_t* words[4];
    const uint64_t* dir[4];
};

// the digit levels t < T of one launch: their matrix levels and outputs
struct wv_digit_set {
    wv_digit_levels lv[WV_MAX_LEVELS];
    uint64_t* out[WV_MAX_LEVELS];
};

// words of the matrix levels 2t of a 4-ary tree (t < T)
struct wv_digit_words {
    const uint64_t* w[WV_MAX_LEVELS / 2];
};

// workgroups of the 2-bit digit kernel (and rows of the zero counts below)
uint64_t wv_digit_blocks(uint64_t n);

// cnt[b * T + t] = zeros in block b of matrix level 2t (blocks of 256 words)
hipError_t wv_digit_zero_counts(const wv_digit_words& a, uint64_t n, uint32_t T, uint32_t* cnt, hipStream_t s);

// the digit strings of digit levels t < T, each in the order of matrix level
// tD (ceil(n*D/64) words; D = 1, 2 or 4), in one launch.  D = 2 takes the zeros before every
// block of level 2t from zpre[b * T + t] (the exclusive scan of the zero
// counts above) and the level's zeros from ztot[t] instead of rank queries;
// D = 4 queries the rank directories in `a`.
hipError_t wv_tree_digits(const wv_digit_set& a, uint32_t T, uint64_t n, uint32_t D, const uint64_t* zpre,
                          const uint64_t* ztot, hipStream_t s);

// ---- runs of balanced trees, derived on the device --------------------------
//
// A balanced tree (binary, or multiary with D-bit digits) over K-bit keys,
// K <= WV_GROUP_MAX_BITS: the run of key prefix g (the top l key bits) on
// binary level l starts, in tree order, after the symbols with a smaller
// prefix, C[g << (K-l)] with C the exclusive prefix of the symbol counts over
// the key space; in the matrix order it starts after the groups whose prefix
// read bit-reversed is smaller (the matrix orders a level by the reversed
// prefix), P[2^l - 1 + brev(g)] - P[2^l - 1] with P the exclusive prefix of
// every level's group counts laid out in bit-reversed order.  No host copy:
// the whole tree build stays ordered on its stream.
constexpr uint32_t WV_GROUP_MAX_BITS = 20;

// workspace of the derivation for K key bits (bytes, 256-aligned pieces)
struct wv_group_ws {
    uint64_t off_cnt, off_C, off_V, off_P, off_part, off_tot, bytes;
};
wv_group_ws wv_group_ws_sizes(uint32_t K);

// C and P from the symbol counts (dev, sigma entries; symbols >= sigma are
// not counted, so C[2^K] < n flags them and the gather below leaves the
// uncovered bits 0)
hipError_t wv_tree_group_runs(const uint64_t* counts, uint32_t sigma, uint32_t K, uint8_t* ws,
                              const wv_group_ws& z, hipStream_t s);

// one tree level of the gather below (passed by value)
struct wv_group_level {
    uint64_t* dst;          // tree level words (in the image)
    const uint64_t* src;    // matrix level words, or the digit string in matrix order (one readable word past the end)
    uint64_t nbits;         // bits on the tree level
    uint16_t* sub;          // multiary: the level's sub-range counters
    uint32_t l;             // binary level of its runs (t * D)
};

// gather every tree level, runs from C and P; with `counts` the levels are
// multiary (D = counts->D bits per symbol) and their counters are taken on the way
hipError_t wv_tree_permute_groups(const wv_group_level* lv, uint32_t nlev, uint32_t K, uint32_t D, const uint8_t* ws,
                                  const wv_group_ws& z, const wv_perm_counts* counts, hipStream_t s);

// gather every tree level (descriptors, runs and tile_seg already on the
// device; tile0 on the host, nlev + 1 entries); with `counts`, the levels are
// multiary and their counters are taken on the way
hipError_t wv_tree_permute(const wv_perm_level* lv_dev, uint32_t nlev, const wv_perm_seg* seg_dev,
                           const uint32_t* tile_seg_dev, const uint32_t* tile0, const wv_perm_counts* counts,
                           hipStream_t s);
