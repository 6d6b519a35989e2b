// wv_common.h -- internal definitions shared by the HIP sources of libwavelet.
//
// The canonical image layout (documented in include/wavelet.h) is computed by
// wv_layout(), callable on the host (planning) and on the device (header
// writer), so the offsets every kernel uses come from one rule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wavelet.h"

#define WV_MAGIC        0x54564157u
#define WV_VERSION      3u
#define WV_HEADER_BYTES 256u
#define WV_LEVEL_BYTES  64u
#define WV_NODE_BYTES   32u     // node record of a binary shaped tree
#define WV_CODE_BYTES   16u
#define WV_SB_BITS      512u    // rank range (superblock), Sec. 5.1
#define WV_SEL_STRIDE   4096u   // select sampling stride, Sec. 5.1
#define WV_SUB_STRIDE   512u    // select sub-sampling stride (second level)
#define WV_XSPAN_LOG2   20u     // sub-ranges spanning 2^20 bits or more keep every answer
#define WV_MAX_LEVELS   32u
#define WV_LEAF         0x80000000u
#define WV_NONE         0xFFFFFFFFu

#define WV_CHECK(call)                                        \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return WT_EHIP;                 \
    } while (0)

__host__ __device__ inline uint64_t wv_round256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }
__host__ __device__ inline uint64_t wv_cdiv(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// L = max(1, ceil(log2 sigma)): the root range is [0, 2^L - 1] (Sec. 2).
__host__ __device__ inline uint32_t wv_key_bits(uint32_t sigma)
{
    uint32_t L = 1;
    while (L < 32 && ((uint64_t)1 << L) < sigma) L++;
    return L;
}

// Sizes of the arrays of one level.
__host__ __device__ inline uint64_t wv_bits_bytes(uint64_t m) { return wv_cdiv(m, 64) * 8; }
__host__ __device__ inline uint64_t wv_rank_bytes(uint64_t m) { return (wv_cdiv(m, WV_SB_BITS) + 1) * 16; }
__host__ __device__ inline uint64_t wv_nsel(uint64_t m) { return wv_cdiv(m, WV_SEL_STRIDE) + 1; }
// Binary levels also keep the position of every one (zero) of ordinal 512j:
// ones at entry j from the front, zeros at entry nsub-1-j from the back,
// unused entries m.  ceil(ones/512) + ceil(zeros/512) <= ceil(m/512) + 1, so
// with one entry more at least one unused entry separates the two halves
// (the end marker of each).  The array follows sel1; the image's level
// record does not hold its offset (it is sel1's end rounded to 256 bytes).
// Levels of D-bit digits: multiary trees, and shaped trees whose codewords
// are D-bit digits (D >= 2; Sec. 4.3 carries shapes over to multiary trees).
__host__ __device__ inline bool wv_multi_levels(uint32_t kind, uint32_t arity_log2)
{
    return kind == WT_KIND_MULTIARY || (kind == WT_KIND_SHAPED && arity_log2 >= 2);
}
// node record of a shaped tree: binary {u64 start, u64 count, u32 child[2],
// u32 level, u32 prefix}; D-bit digits {u64 start, u64 count, u32 level,
// u32 prefix, u32 child[2^D]}
__host__ __device__ inline uint64_t wv_node_bytes(uint32_t arity_log2)
{
    return arity_log2 >= 2 ? 24u + (4ull << arity_log2) : (uint64_t)WV_NODE_BYTES;
}
__host__ __device__ inline uint64_t wv_nsub(uint64_t m) { return wv_cdiv(m, WV_SUB_STRIDE) + 2; }
__host__ __device__ inline uint64_t wv_sub_off(uint64_t sel1_off, uint64_t nsel)
{
    return wv_round256(sel1_off + 8 * nsel);
}
// Clark's rule for long ranges (Sec. 5.1, "Select": a range whose length
// passes a threshold stores the answer of every select in it), applied to
// the sub-ranges between two sub-samples: the ones (zeros) of ordinals
// 512j .. 512j+511 span [p_j, p_{j+1}) with p_{j+1} = m past the last one.
// A sub-range spanning at least 2^20 bits keeps the 512 positions (u32) in
// slot floor(p_j / 2^20) of its kind's pool.  Such sub-ranges are disjoint
// and at least 2^20 long, so two of them never share a slot and a level of m
// bits needs floor(m / 2^20) slots per kind (2 KB each: at most 1/64 of the
// level's bit array per kind).  Pool: the ones' slots, then the zeros'; unused entries m.
__host__ __device__ inline uint64_t wv_nslot(uint64_t m) { return m >> WV_XSPAN_LOG2; }
__host__ __device__ inline uint64_t wv_pool_bytes(uint64_t m) { return wv_nslot(m) * 2 * WV_SUB_STRIDE * 4; }
__host__ __device__ inline uint64_t wv_pool_off(uint64_t sub_off, uint64_t nsub) { return wv_round256(sub_off + 4 * nsub); }
__host__ __device__ inline uint32_t wv_digits_per_word(uint32_t D) { return D == 3 ? 21u : 64u >> (D >> 1); }
// ceil(m / (words * digits per word)); a shift for D = 1, 2, 4 (no 64-bit
// division on the device)
__host__ __device__ inline uint64_t wv_mdiv_words(uint64_t m, uint32_t D, uint32_t words_log2)
{
    if (D == 3) return wv_cdiv(m, (21ull << words_log2));
    const uint32_t sh = words_log2 + 6 - (D >> 1);
    return (m + (1ull << sh) - 1) >> sh;
}
__host__ __device__ inline uint64_t wv_mbits_bytes(uint64_t m, uint32_t D) { return wv_mdiv_words(m, D, 0) * 8; }
// multiary counters: range = 64 words, sub-range = 8 words
__host__ __device__ inline uint64_t wv_mranges(uint64_t m, uint32_t D) { return wv_mdiv_words(m, D, 6); }
__host__ __device__ inline uint64_t wv_msubs(uint64_t m, uint32_t D) { return wv_mdiv_words(m, D, 3); }
__host__ __device__ inline uint64_t wv_mrank_bytes(uint64_t m, uint32_t D)
{
    uint64_t d = 1ull << D;
    return (wv_mranges(m, D) + 1) * d * 8 + wv_msubs(m, D) * d * 2;
}

struct wv_level {
    uint64_t n, bits_off, rank_off, sel0_off, sel1_off, nsel;
    uint64_t sub_off, nsub;   // binary levels: select sub-samples (else 0)
    uint64_t pool_off, nslot; // binary levels: explicit answers of long sub-ranges
};

// Everything needed to place the arrays of an image.
struct wv_layout_in {
    uint32_t kind, arity_log2, nlevels, key_bits;
    uint32_t sigma, pad;
    uint64_t n, nnodes, ncoded;
    uint64_t level_n[WV_MAX_LEVELS];
};

struct wv_layout_out {
    wv_level lv[WV_MAX_LEVELS];
    uint64_t nodes_off, codes_off, image_bytes;
};

__host__ __device__ inline void wv_layout(const wv_layout_in& in, wv_layout_out& out)
{
    const bool multi = wv_multi_levels(in.kind, in.arity_log2);
    const uint32_t D = in.arity_log2;
    uint64_t off = WV_HEADER_BYTES + wv_round256((uint64_t)WV_LEVEL_BYTES * in.nlevels);
    for (uint32_t l = 0; l < in.nlevels; l++) {
        const uint64_t m = in.level_n[l];
        wv_level& L = out.lv[l];
        L.n = m;
        L.bits_off = off;
        off = wv_round256(off + (multi ? wv_mbits_bytes(m, D) : wv_bits_bytes(m)));
        L.rank_off = off;
        off = wv_round256(off + (multi ? wv_mrank_bytes(m, D) : wv_rank_bytes(m)));
        if (!multi) {
            L.nsel = wv_nsel(m);
            L.sel0_off = off;
            off = wv_round256(off + L.nsel * 8);
            L.sel1_off = off;
            off = wv_round256(off + L.nsel * 8);
            L.nsub = wv_nsub(m);
            L.sub_off = off;
            off = wv_round256(off + L.nsub * 4);
            L.nslot = wv_nslot(m);
            L.pool_off = off;
            off = wv_round256(off + wv_pool_bytes(m));
        } else {
            // generalized select: 2^D arrays of nsel samples, digit-major
            L.nsel = wv_nsel(m);
            L.sel0_off = off;
            off = wv_round256(off + (8ull << D) * L.nsel);
            L.sel1_off = 0;
            L.sub_off = L.nsub = 0;
            L.pool_off = L.nslot = 0;
        }
    }
    out.nodes_off = out.codes_off = 0;
    if (in.kind == WT_KIND_SHAPED) {
        out.nodes_off = off;
        off = wv_round256(off + in.nnodes * wv_node_bytes(in.arity_log2));
        out.codes_off = off;
        off = wv_round256(off + (uint64_t)in.sigma * WV_CODE_BYTES);
    }
    out.image_bytes = off;
}

// ---- device helpers ---------------------------------------------------------

// Inclusive scan of one value per lane over the 64 lanes of a wave, in
// registers through DPP lane moves: a scan inside every row of 16 lanes
// (shifts by 1, 2, 4, 8; lanes shifted in from outside the row read 0), then
// the last lane of row 0 added to row 1 and of row 2 to row 3 (broadcast
// 15), then lane 31 added to rows 2 and 3 (broadcast 31).  Every lane of the
// wave must be active.
__device__ inline uint32_t wv_wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// the same for 64-bit values: both halves move, the sum carries
__device__ inline uint64_t wv_wave_incl_scan64(uint64_t v)
{
#define WV_DPP64(ctrl, rows, bound)                                                                  \
    v += ((uint64_t)(uint32_t)__builtin_amdgcn_update_dpp(0, (int)(v >> 32), ctrl, rows, 0xf, bound) << 32) | \
         (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, ctrl, rows, 0xf, bound)
    WV_DPP64(0x111, 0xf, true);
    WV_DPP64(0x112, 0xf, true);
    WV_DPP64(0x114, 0xf, true);
    WV_DPP64(0x118, 0xf, true);
    WV_DPP64(0x142, 0xa, false);
    WV_DPP64(0x143, 0xc, false);
#undef WV_DPP64
    return v;
}

template <typename T>
__device__ inline uint32_t wv_load_sym(const void* S, uint64_t i)
{
    return (uint32_t)((const T*)S)[i];
}

// position of the set bit with 0-based ordinal r in w (r < popcount(w))
__device__ inline uint32_t wv_select_in_word(uint64_t w, uint32_t r)
{
    uint32_t base = 0;
    uint32_t c = __popc((uint32_t)w);
    if (r >= c) { r -= c; w >>= 32; base = 32; }
    uint32_t x = (uint32_t)w;
    for (uint32_t step = 16; step >= 1; step >>= 1) {
        uint32_t lo = x & ((1u << step) - 1u);
        uint32_t cl = __popc(lo);
        if (r >= cl) { r -= cl; x >>= step; base += step; } else { x = lo; }
    }
    return base;
}

// zeros in [0, i) of a binary level, from its rank directory and bit words
__device__ inline uint64_t wv_rank0(const uint64_t* __restrict__ words,
                                    const uint64_t* __restrict__ dir, uint64_t i)
{
    const uint64_t k = i >> 9;
    const uint32_t q = (uint32_t)(i & 511);
    uint64_t r = dir[2 * k];
    const uint32_t j = q >> 6;
    if (j) r += (dir[2 * k + 1] >> (9 * (j - 1))) & 511u;
    const uint32_t t = q & 63;
    if (t) {
        const uint64_t w = words[i >> 6];
        r += t - __popcll(w & ((1ull << t) - 1ull));
    }
    return r;
}

// Position of the b-bit of 0-based ordinal j on a binary level of n bits,
// given the positions p0 of its ordinal 512*floor(j/512) and p1 of the next
// sub-sample (n if none): the rank superblocks between the two are searched
// for the last one with at most j b-bits before it, then its seven relative
// counts give the word.
__device__ inline uint64_t wv_select_dir(const uint64_t* __restrict__ words, const uint64_t* __restrict__ dir,
                                         uint64_t n, uint32_t b, uint64_t j, uint64_t p0, uint64_t p1)
{
    const uint64_t ns = wv_cdiv(n, WV_SB_BITS), nw = wv_cdiv(n, 64);
    uint64_t lo = p0 >> 9, hi = (p1 >> 9) < ns ? (p1 >> 9) : ns - 1;
    auto before = [&](uint64_t k) -> uint64_t { return b ? (k * WV_SB_BITS - dir[2 * k]) : dir[2 * k]; };
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) / 2;
        if (before(mid) <= j) lo = mid; else hi = mid - 1;
    }
    const uint64_t k = lo;
    const uint64_t r = j - before(k);
    const uint64_t blk = dir[2 * k + 1];
    uint32_t qw = 0;
    uint64_t cq = 0;
    for (uint32_t t = 1; t < 8; t++) {
        if (8 * k + t >= nw) break;
        const uint64_t f = (blk >> (9 * (t - 1))) & 511u;
        const uint64_t c = b ? (64u * t - f) : f;
        if (c <= r) { qw = t; cq = c; } else break;
    }
    uint64_t w = words[8 * k + qw];
    if (!b) w = ~w;
    return k * WV_SB_BITS + 64u * qw + wv_select_in_word(w, (uint32_t)(r - cq));
}

// The select samples inside one chunk of nwl words (at most 64 ones and 64
// zeros of ordinal 512k, as a chunk holds 32768 bits), after zex (zeros
// before each word of the chunk) and wds (its words) are in LDS: thread k <
// 128 takes the k-th one of ordinal 512k' in the chunk, thread 128 + k the
// k-th zero; a binary search of zex gives its word, a select inside the word
// its position.  One select per sample instead of a test in every word.
__device__ inline void wv_chunk_samples(const uint64_t* wds, const uint32_t* zex, uint32_t nwl, uint32_t nloc,
                                     uint32_t cw, uint32_t obase, uint32_t zbase, uint32_t ones, uint32_t* sub,
                                     uint32_t nsub, uint64_t* sel0, uint64_t* sel1)
{
    const uint32_t t = threadIdx.x, b = t < 128 ? 1u : 0u, k = t & 127;
    const uint32_t base = b ? obase : zbase, cnt = b ? ones : nloc - ones;
    const uint32_t first = (uint32_t)(wv_cdiv((uint64_t)base, WV_SUB_STRIDE) * WV_SUB_STRIDE - base);   // chunk-local ordinal
    const uint32_t r = first + k * WV_SUB_STRIDE;
    if (r >= cnt || k >= 64) return;
    // b-bits before word w of the chunk
    auto before = [&](uint32_t w) -> uint32_t { return b ? min(64u * w, nloc) - zex[w] : zex[w]; };
    uint32_t lo = 0, hi = nwl - 1;   // the last word with at most r b-bits before it
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (before(mid) <= r) lo = mid; else hi = mid - 1;
    }
    const uint32_t valid = min(64u, nloc - 64u * lo);
    const uint64_t vm = valid >= 64 ? ~0ull : ((1ull << valid) - 1ull);
    const uint64_t x = b ? wds[lo] : (~wds[lo] & vm);
    const uint32_t p = 64 * (cw + lo) + wv_select_in_word(x, r - before(lo));
    const uint32_t ord = base + r;
    if (b) {
        sub[ord / WV_SUB_STRIDE] = p;
        if (ord % WV_SEL_STRIDE == 0) sel1[ord / WV_SEL_STRIDE] = p;
    } else {
        sub[nsub - 1 - ord / WV_SUB_STRIDE] = p;
        if (ord % WV_SEL_STRIDE == 0) sel0[ord / WV_SEL_STRIDE] = p;
    }
}

// A binary level whose explicit answers are written by wv_xsel_block: the
// image, the level's length and array offsets, and the first workgroup of
// the level in the launch (2 * nslot workgroups per level).
struct wv_xlevel {
    uint8_t* image;
    uint64_t m, bits_off, rank_off, sub_off, nsub;
    uint32_t blk0, pad;
};

// One slot of a level's pool, by a workgroup of WV_SUB_STRIDE threads:
// local = kind * nslot + slot, ones (kind 0 here) first.  The only sub-range
// that can own slot s is the last one starting before lim = (s+1)*2^20: with
// c b-bits before lim (one rank directory entry, lim being a multiple of
// 512 and at most m), it is j = (c-1)/512.  It owns the slot if it starts
// at s*2^20 or later and spans 2^20 bits or more.  Thread t then writes the
// position of ordinal 512j+t (found by the directory search), or m past the
// kind's count and in an unowned slot.
__device__ inline void wv_xsel_block(const wv_xlevel& X, uint32_t local)
{
    const uint64_t m = X.m, nslot = wv_nslot(m), ns = wv_cdiv(m, WV_SB_BITS);
    const uint32_t b = local < nslot ? 1u : 0u;
    const uint64_t slot = b ? local : local - nslot;
    const uint64_t* dir = (const uint64_t*)(X.image + X.rank_off);
    const uint64_t* words = (const uint64_t*)(X.image + X.bits_off);
    const uint32_t* sub = (const uint32_t*)(X.image + X.sub_off);
    uint32_t* pool = (uint32_t*)(X.image + wv_pool_off(X.sub_off, X.nsub)) +
                     ((b ? 0 : nslot) + slot) * WV_SUB_STRIDE;
    const uint64_t zeros = dir[2 * ns], count = b ? m - zeros : zeros;
    const uint64_t J = wv_cdiv(count, WV_SUB_STRIDE);   // sub-ranges of the kind
    auto entry = [&](uint64_t j) -> uint64_t { return b ? sub[j] : sub[X.nsub - 1 - j]; };
    const uint64_t lim = (slot + 1) << WV_XSPAN_LOG2;
    const uint64_t zb = dir[2 * (lim >> 9)];
    const uint64_t c = b ? lim - zb : zb;
    uint64_t out = m;
    if (c) {
        const uint64_t j = (c - 1) / WV_SUB_STRIDE;   // j < J
        const uint64_t p0 = entry(j);
        const uint64_t p1 = j + 1 < J ? entry(j + 1) : m;
        const uint64_t o = j * WV_SUB_STRIDE + threadIdx.x;
        if (p0 >= (slot << WV_XSPAN_LOG2) && p1 - p0 >= (1ull << WV_XSPAN_LOG2) && o < count)
            out = wv_select_dir(words, dir, m, b, o, p0, p1);
    }
    pool[threadIdx.x] = (uint32_t)out;
}

// the low bit of every digit equal to g among the first t (< P) digits of
// word w (bit D*i for digit i)
__device__ inline uint64_t wv_digit_mask(uint64_t w, uint32_t D, uint32_t g, uint32_t t)
{
    if (t == 0) return 0;
    // low-bit-of-every-digit mask: bits 0, D, 2D, ... of the P = 64/D digits
    // (D = 1..4; a constant per width, no division)
    const uint64_t lowm = D == 1 ? ~0ull : D == 2 ? 0x5555555555555555ull
                        : D == 3 ? 0x1249249249249249ull : 0x1111111111111111ull;
    uint64_t pat = lowm * (uint64_t)g;
    uint64_t x = w ^ pat;               // digit == g  <=>  digit of x == 0
    uint64_t any = x;
    for (uint32_t b = 1; b < D; b++) any |= x >> b;
    uint64_t eq = ~any & lowm;
    uint64_t keep = (t * D >= 64) ? ~0ull : ((1ull << (t * D)) - 1ull);
    return eq & keep;
}

// number of digits equal to g among the first t (< P) digits of word w
__device__ inline uint32_t wv_count_digit(uint64_t w, uint32_t D, uint32_t g, uint32_t t)
{
    return (uint32_t)__popcll(wv_digit_mask(w, D, g, t));
}

// index of the digit of value g with 0-based ordinal j in word w (j below
// the word's count of g among its first t digits)
__device__ inline uint32_t wv_digit_select(uint64_t w, uint32_t D, uint32_t g, uint32_t t, uint32_t j)
{
    const uint32_t b = wv_select_in_word(wv_digit_mask(w, D, g, t), j);
    return D == 1 ? b : (D == 2 ? b >> 1 : (D == 4 ? b >> 2 : b / 3u));
}

// digit g count in [0, i) of a multiary level from its counters and words
__device__ inline uint64_t wv_mrank(const uint64_t* __restrict__ words, const uint8_t* __restrict__ cnt,
                                    uint64_t m, uint32_t D, uint32_t g, uint64_t i)
{
    const uint32_t P = wv_digits_per_word(D);
    const uint64_t d = 1ull << D;
    const uint64_t nr = wv_mranges(m, D);
    const uint64_t* rng = (const uint64_t*)cnt;
    const uint16_t* sub = (const uint16_t*)(cnt + (nr + 1) * d * 8);
    const uint64_t rk = i / (64ull * P);
    uint64_t r = rng[rk * d + g];
    // the sub-range holding i; for i = m at a sub-range boundary inside the
    // last range there is no such sub-range, and the words are counted from
    // the range start
    const uint64_t sk = i / (8ull * P);
    uint64_t w0 = rk * 64;
    if (sk < wv_msubs(m, D)) {
        r += sub[sk * d + g];
        w0 = sk * 8;
    }
    const uint64_t wk = i / P;
    // whole words between the (sub-)range start and the word holding i
    for (uint64_t w = w0; w < wk; w++) r += wv_count_digit(words[w], D, g, P);
    const uint32_t t = (uint32_t)(i - wk * P);
    if (t) r += wv_count_digit(words[wk], D, g, t);
    return r;
}


// Generalized select on a multiary level (Sec. 5.2, "Select"): position of
// the digit g of 0-based ordinal o (o below the level's count of g).  The
// digit's sample of ordinal 4096*floor(o/4096) and the next one bound the
// 64-word ranges to search (binary search on the range counters), then the
// sub-range counters and the words of one sub-range give the position.
__device__ inline uint64_t wv_mselect(const uint64_t* __restrict__ words, const uint8_t* __restrict__ cnt,
                                      const uint64_t* __restrict__ sel, uint64_t nsel, uint64_t m, uint32_t D,
                                      uint32_t g, uint64_t o)
{
    const uint32_t P = wv_digits_per_word(D);
    const uint64_t d = 1ull << D;
    const uint64_t nr = wv_mranges(m, D), nsub = wv_msubs(m, D);
    const uint64_t* rng = (const uint64_t*)cnt;
    const uint16_t* sub = (const uint16_t*)(cnt + (nr + 1) * d * 8);
    const uint64_t k = o / WV_SEL_STRIDE;
    const uint64_t p0 = sel[g * nsel + k], p1 = sel[g * nsel + k + 1];
    const uint64_t RD = 64ull * P;   // digits per range
    uint64_t lo = p0 / RD, hi = p1 >= m ? nr - 1 : p1 / RD;
    while (lo < hi) {   // the last range starting with at most o digits g before it
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (rng[mid * d + g] <= o) lo = mid; else hi = mid - 1;
    }
    uint64_t before = rng[lo * d + g];
    uint64_t w = lo * 64;
    for (uint64_t sk = lo * 8 + 1; sk < lo * 8 + 8 && sk < nsub; sk++) {
        const uint64_t b = rng[lo * d + g] + sub[sk * d + g];
        if (b > o) break;
        before = b;
        w = sk * 8;
    }
    const uint64_t nw = wv_cdiv(m, P);
    for (;; w++) {   // the word holding it is at most 7 words on
        const uint32_t t = (uint32_t)min<uint64_t>(P, m - w * P);
        const uint32_t c = wv_count_digit(words[w], D, g, t);
        if (before + c > o || w + 1 >= nw) return w * P + wv_digit_select(words[w], D, g, t, (uint32_t)(o - before));
        before += c;
    }
}
