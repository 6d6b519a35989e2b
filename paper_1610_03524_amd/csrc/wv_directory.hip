// wv_directory.hip -- rank/select directories, multiary counters, image
// header and input validation.
//
// Binary levels (Sec. 5.1, "Rank"): the ones of every 512-bit superblock are
// counted, an exclusive prefix sum gives the rank at every superblock
// boundary (the paper's prefix sum over per-word counts, read every 8th
// word), and each superblock then writes {zeros before it, seven 9-bit zero
// counts relative to its start}.  Sampled select (Sec. 5.1, "Select"): the
// superblock holding the one (zero) of ordinal 4096k finds it inside its
// word and writes its position; the same for ordinals 512k into the
// sub-sample array (the second sampling level of Clark's structure, so that
// a select searches the ranges between two positions 512 ones apart); a
// sub-range spanning 2^20 bits or more then gets all its answers stored in
// the level's pool (Clark's rule for long ranges).
// Multiary levels (Sec. 5.2, "Rank"): the same with one counter per digit
// value.
#include <algorithm>

#include "wv_internal.h"

namespace {

constexpr int DIR_THREADS = 256;

__device__ inline uint64_t valid_mask(int64_t vb)
{
    if (vb <= 0) return 0ull;
    if (vb >= 64) return ~0ull;
    return (1ull << vb) - 1ull;
}

__global__ void __launch_bounds__(DIR_THREADS)
count_superblocks_k(const uint64_t* __restrict__ words, uint64_t n, uint32_t* __restrict__ sb_ones)
{
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t ns = wv_cdiv(n, WV_SB_BITS), nw = wv_cdiv(n, 64);
    if (k >= ns) return;
    uint32_t c = 0;
    for (uint64_t j = 0; j < 8; j++) {
        uint64_t w = 8 * k + j;
        if (w < nw) c += __popcll(words[w]);
    }
    sb_ones[k] = c;
}

__global__ void __launch_bounds__(DIR_THREADS)
dir_write_k(uint8_t* __restrict__ image, wv_level L, const uint64_t* __restrict__ sb_pre)
{
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t n = L.n;
    const uint64_t ns = wv_cdiv(n, WV_SB_BITS), nw = wv_cdiv(n, 64);
    if (k >= ns) return;
    const uint64_t* words = (const uint64_t*)(image + L.bits_off);
    uint64_t* dir = (uint64_t*)(image + L.rank_off);
    uint64_t* sel0 = (uint64_t*)(image + L.sel0_off);
    uint64_t* sel1 = (uint64_t*)(image + L.sel1_off);
    const uint64_t base = k * WV_SB_BITS;
    const uint64_t ones_before = sb_pre[k];
    const uint64_t zeros_before = base - ones_before;

    uint64_t w[8];
    uint32_t o[8], z[8];
    uint64_t blk = 0;
    uint32_t zacc = 0, oacc = 0;
    for (int j = 0; j < 8; j++) {
        const uint64_t wi = 8 * k + j;
        w[j] = wi < nw ? words[wi] : 0ull;
        const int64_t vb = (int64_t)n - (int64_t)(base + 64u * j);
        const uint32_t v = vb <= 0 ? 0u : (vb >= 64 ? 64u : (uint32_t)vb);
        o[j] = __popcll(w[j]);
        z[j] = v - o[j];
        if (j >= 1) blk |= (uint64_t)zacc << (9 * (j - 1));
        zacc += z[j];
        oacc += o[j];
    }
    dir[2 * k] = zeros_before;
    dir[2 * k + 1] = blk;

    // the one of ordinal t (a multiple of 512) inside this superblock (a
    // superblock holds at most one), a sample when t is a multiple of 4096
    uint32_t* sub = (uint32_t*)(image + L.sub_off);
    uint64_t t = wv_cdiv(ones_before, WV_SUB_STRIDE) * WV_SUB_STRIDE;
    if (t < ones_before + oacc) {
        uint32_t r = (uint32_t)(t - ones_before);
        for (int j = 0; j < 8; j++) {
            if (r < o[j]) {
                const uint64_t p = base + 64u * j + wv_select_in_word(w[j], r);
                sub[t / WV_SUB_STRIDE] = (uint32_t)p;
                if (t % WV_SEL_STRIDE == 0) sel1[t / WV_SEL_STRIDE] = p;
                break;
            }
            r -= o[j];
        }
    }
    t = wv_cdiv(zeros_before, WV_SUB_STRIDE) * WV_SUB_STRIDE;
    if (t < zeros_before + zacc) {
        uint32_t r = (uint32_t)(t - zeros_before);
        for (int j = 0; j < 8; j++) {
            if (r < z[j]) {
                const int64_t vb = (int64_t)n - (int64_t)(base + 64u * j);
                const uint64_t p = base + 64u * j + wv_select_in_word(~w[j] & valid_mask(vb), r);
                sub[L.nsub - 1 - t / WV_SUB_STRIDE] = (uint32_t)p;
                if (t % WV_SEL_STRIDE == 0) sel0[t / WV_SEL_STRIDE] = p;
                break;
            }
            r -= z[j];
        }
    }
}

__global__ void __launch_bounds__(DIR_THREADS)
dir_finish_k(uint8_t* __restrict__ image, uint32_t level, wv_level L,
             const uint64_t* __restrict__ total_ones, uint64_t* __restrict__ zl_dev)
{
    const uint64_t n = L.n;
    const uint64_t ones = *total_ones, zeros = n - ones;
    const uint64_t ns = wv_cdiv(n, WV_SB_BITS);
    uint64_t* dir = (uint64_t*)(image + L.rank_off);
    uint64_t* sel0 = (uint64_t*)(image + L.sel0_off);
    uint64_t* sel1 = (uint64_t*)(image + L.sel1_off);
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        dir[2 * ns] = zeros;
        dir[2 * ns + 1] = 0;
        uint64_t* desc = (uint64_t*)(image + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * level);
        desc[1] = zeros;
        desc[2] = ones;
        if (zl_dev) *zl_dev = zeros;
    }
    for (uint64_t k = wv_cdiv(ones, WV_SEL_STRIDE) + tid; k < L.nsel; k += stride) sel1[k] = n;
    for (uint64_t k = wv_cdiv(zeros, WV_SEL_STRIDE) + tid; k < L.nsel; k += stride) sel0[k] = n;
    // sub-samples between the ones' and the zeros' entries
    uint32_t* sub = (uint32_t*)(image + L.sub_off);
    const uint64_t sub_hi = L.nsub - wv_cdiv(zeros, WV_SUB_STRIDE);
    for (uint64_t k = wv_cdiv(ones, WV_SUB_STRIDE) + tid; k < sub_hi; k += stride) sub[k] = (uint32_t)n;
}

// ---- multiary counters -------------------------------------------------------

// Multiary counters of M levels at once (level t = blockIdx.y, m[t] digits),
// one wave per range of 64 words (lane = word).  Range counts and prefixes
// are laid out [range][level][digit] with nr0 rows, the ranges of the
// longest level (a shorter level counts zero in the rows past its end).
struct MLevels {
    uint64_t bits_off[WV_MAX_LEVELS], rank_off[WV_MAX_LEVELS], sel_off[WV_MAX_LEVELS];
    uint64_t m[WV_MAX_LEVELS], nsel[WV_MAX_LEVELS];
    uint64_t nr0, nsel0;   // most ranges, most samples per digit of any level
    uint32_t M, D;
};

// Generalized select samples (Sec. 5.2, "Select"): every digit value's
// occurrences of ordinal 4096k, found from the finished range counters: one
// wave per 64-word range, which holds at most one sample of each value (a
// range has at most 64 * 64 digits); lane = word.
__global__ void __launch_bounds__(DIR_THREADS)
msel_k(uint8_t* __restrict__ image, MLevels a)
{
    const uint32_t lane = threadIdx.x & 63, t = blockIdx.y;
    const uint64_t r = ((uint64_t)blockIdx.x * DIR_THREADS + threadIdx.x) >> 6;
    const uint32_t D = a.D, P = wv_digits_per_word(D), d = 1u << D;
    const uint64_t m = a.m[t], nr = wv_mranges(m, D), nw = wv_cdiv(m, P);
    if (r >= nr) return;   // whole waves: the scans below need every lane
    const uint64_t* words = (const uint64_t*)(image + a.bits_off[t]);
    const uint64_t* rng = (const uint64_t*)(image + a.rank_off[t]);
    uint64_t* sel = (uint64_t*)(image + a.sel_off[t]);
    const uint64_t wi = 64 * r + lane;
    const uint64_t w = wi < nw ? words[wi] : 0ull;
    const uint32_t c = wi < nw ? (uint32_t)min<uint64_t>(P, m - wi * P) : 0u;
    for (uint32_t g = 0; g < d; g++) {
        const uint32_t v = wv_count_digit(w, D, g, c);
        const uint32_t inc = wv_wave_incl_scan(v);
        const uint64_t base = rng[r * d + g];                          // digits g before the range
        const uint64_t o = wv_cdiv(base, WV_SEL_STRIDE) * WV_SEL_STRIDE;   // the next sampled ordinal
        if (o >= base + inc - v && o < base + inc)
            sel[g * a.nsel[t] + o / WV_SEL_STRIDE] = wi * P + wv_digit_select(w, D, g, c, (uint32_t)(o - (base + inc - v)));
    }
}

// samples past each value's last one: the level length
__global__ void __launch_bounds__(DIR_THREADS)
msel_fill_k(uint8_t* __restrict__ image, MLevels a)
{
    const uint32_t t = blockIdx.y, d = 1u << a.D;
    const uint64_t m = a.m[t], nsel = a.nsel[t], nr = wv_mranges(m, a.D);
    const uint64_t* rng = (const uint64_t*)(image + a.rank_off[t]);
    uint64_t* sel = (uint64_t*)(image + a.sel_off[t]);
    for (uint64_t i = (uint64_t)blockIdx.x * DIR_THREADS + threadIdx.x; i < d * nsel; i += (uint64_t)gridDim.x * DIR_THREADS) {
        const uint64_t g = i / nsel, k = i % nsel;
        if (k >= wv_cdiv(rng[nr * d + g], WV_SEL_STRIDE)) sel[i] = m;
    }
}

hipError_t launch_msel(uint8_t* image, const MLevels& a, hipStream_t s)
{
    const uint64_t nr = a.nr0;
    const uint64_t d = 1ull << a.D;
    if (nr) msel_k<<<dim3((uint32_t)wv_cdiv(nr, DIR_THREADS / 64), a.M), DIR_THREADS, 0, s>>>(image, a);
    msel_fill_k<<<dim3((uint32_t)std::min<uint64_t>(wv_cdiv(d * a.nsel0, DIR_THREADS), 1024), a.M), DIR_THREADS, 0, s>>>(
        image, a);
    return hipGetLastError();
}

__global__ void __launch_bounds__(DIR_THREADS)
mcount_k(const uint8_t* __restrict__ image, MLevels a, uint32_t* __restrict__ rng_cnt)
{
    const uint32_t lane = threadIdx.x & 63, t = blockIdx.y;
    const uint64_t r = ((uint64_t)blockIdx.x * DIR_THREADS + threadIdx.x) >> 6;
    const uint32_t D = a.D, P = wv_digits_per_word(D), d = 1u << D;
    const uint64_t m = a.m[t], nw = wv_cdiv(m, P);
    // every row of the counts: rows past the level's end count zero
    if (r >= a.nr0) return;   // whole waves: the scans below need every lane
    const uint64_t* words = (const uint64_t*)(image + a.bits_off[t]);
    const uint64_t wi = 64 * r + lane;
    const uint64_t w = wi < nw ? words[wi] : 0ull;
    const uint32_t c = wi < nw ? (uint32_t)min<uint64_t>(P, m - wi * P) : 0u;
    for (uint32_t g = 0; g < d; g++) {
        const uint32_t inc = wv_wave_incl_scan(wv_count_digit(w, D, g, c));
        if (lane == 63) rng_cnt[(r * a.M + t) * d + g] = inc;
    }
}

__global__ void __launch_bounds__(DIR_THREADS)
mwrite_k(uint8_t* __restrict__ image, MLevels a, const uint64_t* __restrict__ rng_pre)
{
    const uint32_t lane = threadIdx.x & 63, t = blockIdx.y;
    const uint64_t r = ((uint64_t)blockIdx.x * DIR_THREADS + threadIdx.x) >> 6;
    const uint32_t D = a.D, P = wv_digits_per_word(D), d = 1u << D;
    const uint64_t m = a.m[t], nr = wv_mranges(m, D), nsub = wv_msubs(m, D), nw = wv_cdiv(m, P);
    if (r >= nr) return;   // whole waves
    const uint64_t* words = (const uint64_t*)(image + a.bits_off[t]);
    uint64_t* rng = (uint64_t*)(image + a.rank_off[t]);
    uint16_t* sub = (uint16_t*)(image + a.rank_off[t] + (nr + 1) * d * 8);
    if (lane < d) rng[r * d + lane] = rng_pre[(r * a.M + t) * d + lane];
    const uint64_t wi = 64 * r + lane;
    const uint64_t w = wi < nw ? words[wi] : 0ull;
    const uint32_t c = wi < nw ? (uint32_t)min<uint64_t>(P, m - wi * P) : 0u;
    // a sub-range of 8 words stores every digit's count from the range start
    const uint64_t sk = 8 * r + (lane >> 3);
    for (uint32_t g = 0; g < d; g++) {
        const uint32_t v = wv_count_digit(w, D, g, c);
        const uint32_t ex = wv_wave_incl_scan(v) - v;
        if ((lane & 7) == 0 && sk < nsub) sub[sk * d + g] = (uint16_t)ex;
    }
}

// range counters from the scanned range counts (one thread per entry)
__global__ void __launch_bounds__(DIR_THREADS)
mrange_k(uint8_t* __restrict__ image, MLevels a, const uint64_t* __restrict__ rng_pre)
{
    const uint32_t t = blockIdx.y, d = 1u << a.D;
    const uint64_t i = (uint64_t)blockIdx.x * DIR_THREADS + threadIdx.x;
    const uint64_t nr = wv_mranges(a.m[t], a.D);
    if (i >= nr * d) return;
    uint64_t* rng = (uint64_t*)(image + a.rank_off[t]);
    rng[i] = rng_pre[((i / d) * a.M + t) * d + i % d];
}

__global__ void mfinish_k(uint8_t* __restrict__ image, MLevels a, const uint64_t* __restrict__ totals)
{
    const uint32_t t = blockIdx.x, d = 1u << a.D;
    const uint64_t nr = wv_mranges(a.m[t], a.D);
    uint64_t* rng = (uint64_t*)(image + a.rank_off[t]);
    if (threadIdx.x < d) rng[nr * d + threadIdx.x] = totals[t * d + threadIdx.x];
}

// ---- header ------------------------------------------------------------------

// 8-byte aligned middle in words, the ends in bytes
__device__ inline void zero_bytes(uint8_t* img, uint64_t lo, uint64_t hi)
{
    if (lo >= hi) return;
    const uint64_t wlo = min(hi, (lo + 7) & ~7ull), whi = max(wlo, hi & ~7ull);
    for (uint64_t b = lo; b < wlo; b++) img[b] = 0;
    for (uint64_t w = wlo / 8; w < whi / 8; w++) ((uint64_t*)img)[w] = 0;
    for (uint64_t b = whi; b < hi; b++) img[b] = 0;
}

// The header, the level records and every gap between consecutive arrays
// (arrays start on 256-byte boundaries, so each gap is under 256 bytes).
// The layout comes from the host; thread l < nlevels writes level l's record
// and the gaps after its arrays, thread nlevels the header and the gaps
// around it and after the node and codeword tables: no thread waits for
// another.
__global__ void __launch_bounds__(64)
header_k(uint8_t* __restrict__ img, wv_layout_in in, wv_layout_out lay)
{
    const uint32_t t = threadIdx.x, nl = in.nlevels, D = in.arity_log2;
    const bool multi = wv_multi_levels(in.kind, in.arity_log2), shaped = in.kind == WT_KIND_SHAPED;
    const uint64_t after_levels = shaped ? lay.nodes_off : lay.image_bytes;
    if (t < nl) {
        const wv_level& L = lay.lv[t];
        const uint64_t next = t + 1 < nl ? lay.lv[t + 1].bits_off : after_levels;
        zero_bytes(img, L.bits_off + (multi ? wv_mbits_bytes(L.n, D) : wv_bits_bytes(L.n)), L.rank_off);
        zero_bytes(img, L.rank_off + (multi ? wv_mrank_bytes(L.n, D) : wv_rank_bytes(L.n)), L.sel0_off);
        if (multi) {
            zero_bytes(img, L.sel0_off + (8ull << D) * L.nsel, next);
        } else {
            zero_bytes(img, L.sel0_off + 8 * L.nsel, L.sel1_off);
            zero_bytes(img, L.sel1_off + 8 * L.nsel, L.sub_off);
            zero_bytes(img, L.sub_off + 4 * L.nsub, L.pool_off);
            zero_bytes(img, L.pool_off + wv_pool_bytes(L.n), next);
        }
        uint64_t* e = (uint64_t*)(img + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * t);
        e[0] = L.n;
        e[1] = 0;
        e[2] = 0;
        e[3] = L.bits_off;
        e[4] = L.rank_off;
        e[5] = L.sel0_off;
        e[6] = L.sel1_off;
        e[7] = L.nsel;
    } else if (t == nl) {
        uint32_t* h32 = (uint32_t*)img;
        uint64_t* h64 = (uint64_t*)img;
        h32[0] = WV_MAGIC;
        h32[1] = WV_VERSION;
        h32[2] = in.kind;
        h32[3] = in.arity_log2;
        h64[2] = in.n;
        h32[6] = in.sigma;
        h32[7] = in.nlevels;
        h32[8] = in.key_bits;
        h32[9] = 0;
        h64[5] = lay.image_bytes;
        h64[6] = WV_HEADER_BYTES;
        h64[7] = lay.nodes_off;
        h64[8] = in.nnodes;
        h64[9] = lay.codes_off;
        h64[10] = in.ncoded;
        zero_bytes(img, 88, WV_HEADER_BYTES);
        zero_bytes(img, WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * nl, nl ? lay.lv[0].bits_off : after_levels);
        if (shaped) {
            zero_bytes(img, lay.nodes_off + in.nnodes * wv_node_bytes(in.arity_log2), lay.codes_off);
            zero_bytes(img, lay.codes_off + (uint64_t)in.sigma * WV_CODE_BYTES, lay.image_bytes);
        }
    }
}

// ---- validation / symbol counts ------------------------------------------------

constexpr uint32_t LDS_HIST_MAX = 8192;

// Symbols checked against sigma and counted (an LDS histogram per workgroup
// when sigma is small).  The input is read in 16-byte pieces, four in flight
// per thread, when it is 16-byte aligned; the rest symbol by symbol.
template <typename T>
__global__ void __launch_bounds__(DIR_THREADS)
validate_k(const void* __restrict__ S, uint64_t n, uint32_t sigma, uint32_t* __restrict__ status,
           unsigned long long* __restrict__ counts)
{
    __shared__ uint32_t h[LDS_HIST_MAX];
    const bool lds = counts && sigma <= LDS_HIST_MAX;
    if (lds) {
        for (uint32_t b = threadIdx.x; b < sigma; b += blockDim.x) h[b] = 0;
        __syncthreads();
    }
    bool bad = false;
    auto take = [&](uint32_t x) {
        if (x >= sigma) bad = true;
        else if (lds) atomicAdd(&h[x], 1u);
        else if (counts) atomicAdd(&counts[x], 1ull);
    };
    auto take16 = [&](const uint4& v) {
        const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (sizeof(T) == 4) {
                take(q[k]);
            } else if (sizeof(T) == 2) {
                take(q[k] & 0xFFFFu);
                take(q[k] >> 16);
            } else {
#pragma unroll
                for (int b = 0; b < 4; b++) take((q[k] >> (8 * b)) & 0xFFu);
            }
        }
    };
    constexpr uint32_t PER = 16 / sizeof(T);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nv = ((uintptr_t)S & 15u) == 0 ? n / PER : 0;   // whole 16-byte pieces
    const uint4* __restrict__ S4 = (const uint4*)S;
    uint64_t i = t0;
    for (; i + 3 * stride < nv; i += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = S4[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; u++) take16(v[u]);
    }
    for (; i < nv; i += stride) take16(S4[i]);
    for (uint64_t k = nv * PER + t0; k < n; k += stride) take(wv_load_sym<T>(S, k));
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0 && status) atomicOr(status, 1u);
    if (lds) {
        __syncthreads();
        for (uint32_t b = threadIdx.x; b < sigma; b += blockDim.x)
            if (h[b]) atomicAdd(&counts[b], (unsigned long long)h[b]);
    }
}

// explicit select answers of the long sub-ranges of up to WV_MAX_LEVELS
// binary levels of one image (after their directories and sub-samples)
struct XList {
    wv_xlevel lv[WV_MAX_LEVELS];
    uint32_t n;
};

__global__ void __launch_bounds__(WV_SUB_STRIDE)
xsel_k(XList a)
{
    uint32_t i = 0;
    while (i + 1 < a.n && a.lv[i + 1].blk0 <= blockIdx.x) i++;
    wv_xsel_block(a.lv[i], blockIdx.x - a.lv[i].blk0);
}

hipError_t launch_xsel(uint8_t* image, const wv_level* lv, uint32_t nl, hipStream_t s)
{
    XList a{};
    uint32_t blocks = 0;
    for (uint32_t l = 0; l < nl; l++) {
        const uint64_t nslot = wv_nslot(lv[l].n);
        if (!nslot) continue;
        wv_xlevel& x = a.lv[a.n++];
        x.image = image;
        x.m = lv[l].n;
        x.bits_off = lv[l].bits_off;
        x.rank_off = lv[l].rank_off;
        x.sub_off = lv[l].sub_off;
        x.nsub = lv[l].nsub;
        x.blk0 = blocks;
        blocks += (uint32_t)(2 * nslot);
    }
    if (!blocks) return hipSuccess;
    xsel_k<<<blocks, WV_SUB_STRIDE, 0, s>>>(a);
    return hipGetLastError();
}

__global__ void fill_u64_k(uint64_t* p, uint64_t count, uint64_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

inline uint32_t grid_for(uint64_t items, uint32_t threads, uint32_t cap = 65535u)
{
    uint64_t g = wv_cdiv(items ? items : 1, threads);
    return (uint32_t)(g < cap ? g : cap);
}

}  // namespace

hipError_t wv_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s)
{
    if (!count) return hipSuccess;
    fill_u64_k<<<grid_for(count, 256, 4096), 256, 0, s>>>(p, count, value);
    return hipGetLastError();
}

hipError_t wv_count_superblocks(const uint8_t* image, const wv_level& L, uint32_t* sb_ones, hipStream_t s)
{
    const uint64_t ns = wv_cdiv(L.n, WV_SB_BITS);
    if (!ns) return hipSuccess;
    count_superblocks_k<<<(uint32_t)wv_cdiv(ns, DIR_THREADS), DIR_THREADS, 0, s>>>(
        (const uint64_t*)(image + L.bits_off), L.n, sb_ones);
    return hipGetLastError();
}

hipError_t wv_binary_directory(uint8_t* image, uint32_t level, const wv_level& L,
                               const wv_dir_scratch& sc, uint64_t* zl_dev, hipStream_t s)
{
    const uint64_t ns = wv_cdiv(L.n, WV_SB_BITS);
    hipError_t e = wv_scan_u32(sc.sb_ones, sc.sb_pre, ns, 1, sc.partial, sc.total, s);
    if (e != hipSuccess) return e;
    if (ns) dir_write_k<<<(uint32_t)wv_cdiv(ns, DIR_THREADS), DIR_THREADS, 0, s>>>(image, L, sc.sb_pre);
    dir_finish_k<<<grid_for(L.nsel, DIR_THREADS, 64), DIR_THREADS, 0, s>>>(image, level, L, sc.total, zl_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_xsel(image, &L, 1, s);
}

static MLevels mlevels(const wv_level* lv, uint32_t M, uint32_t D)
{
    MLevels a{};
    a.M = M;
    a.D = D;
    for (uint32_t t = 0; t < M; t++) {
        a.bits_off[t] = lv[t].bits_off;
        a.rank_off[t] = lv[t].rank_off;
        a.sel_off[t] = lv[t].sel0_off;
        a.m[t] = lv[t].n;
        a.nsel[t] = lv[t].nsel;
        a.nr0 = std::max<uint64_t>(a.nr0, wv_mranges(lv[t].n, D));
        a.nsel0 = std::max<uint64_t>(a.nsel0, lv[t].nsel);
    }
    return a;
}

hipError_t wv_multiary_counters(uint8_t* image, const wv_level* lv, uint32_t M, uint32_t D,
                                const wv_mdir_scratch& sc, hipStream_t s)
{
    if (!M) return hipSuccess;
    const MLevels a = mlevels(lv, M, D);
    const uint64_t nr = a.nr0;
    const uint32_t d = 1u << D;
    const dim3 grid((uint32_t)wv_cdiv(nr, DIR_THREADS / 64), M);
    if (nr) mcount_k<<<grid, DIR_THREADS, 0, s>>>(image, a, sc.rng_cnt);
    hipError_t e = wv_scan_u32(sc.rng_cnt, sc.rng_pre, nr, M * d, sc.partial, sc.totals, s);
    if (e != hipSuccess) return e;
    if (nr) mwrite_k<<<grid, DIR_THREADS, 0, s>>>(image, a, sc.rng_pre);
    mfinish_k<<<M, 64, 0, s>>>(image, a, sc.totals);
    return launch_msel(image, a, s);
}

hipError_t wv_multiary_ranges(uint8_t* image, const wv_level* lv, uint32_t M, uint32_t D,
                              const wv_mdir_scratch& sc, hipStream_t s)
{
    if (!M) return hipSuccess;
    const MLevels a = mlevels(lv, M, D);
    const uint64_t nr = a.nr0;
    const uint32_t d = 1u << D;
    hipError_t e = wv_scan_u32(sc.rng_cnt, sc.rng_pre, nr, M * d, sc.partial, sc.totals, s);
    if (e != hipSuccess) return e;
    if (nr) mrange_k<<<dim3((uint32_t)wv_cdiv(nr * d, DIR_THREADS), M), DIR_THREADS, 0, s>>>(image, a, sc.rng_pre);
    mfinish_k<<<M, 64, 0, s>>>(image, a, sc.totals);
    return launch_msel(image, a, s);
}

hipError_t wv_write_header(uint8_t* image, const wv_layout_in& in, hipStream_t s)
{
    wv_layout_out lay;
    wv_layout(in, lay);
    header_k<<<1, 64, 0, s>>>(image, in, lay);
    return hipGetLastError();
}

hipError_t wv_validate(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma,
                       uint8_t* image, uint64_t* counts, hipStream_t s)
{
    uint32_t* status = image ? (uint32_t*)(image + 36) : nullptr;
    unsigned long long* c = (unsigned long long*)counts;
    if (counts) {
        hipError_t e = wv_fill_u64(counts, sigma, 0, s);
        if (e != hipSuccess) return e;
    }
    if (!n) return hipSuccess;
    const uint32_t grid = grid_for(n, DIR_THREADS * 64, 1024);
    if (sym_bytes == 1) validate_k<uint8_t><<<grid, DIR_THREADS, 0, s>>>(S, n, sigma, status, c);
    else if (sym_bytes == 2) validate_k<uint16_t><<<grid, DIR_THREADS, 0, s>>>(S, n, sigma, status, c);
    else validate_k<uint32_t><<<grid, DIR_THREADS, 0, s>>>(S, n, sigma, status, c);
    return hipGetLastError();
}

namespace {

// status bit 1 when a symbol's count differs from the one the shape gave
__global__ void counts_match_k(const uint64_t* __restrict__ got, const uint64_t* __restrict__ want, uint32_t sigma,
                               uint32_t* __restrict__ status)
{
    bool bad = false;
    // 64-bit index: sigma may lie within one stride of 2^32
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < sigma; x += (uint64_t)gridDim.x * blockDim.x)
        bad |= got[x] != want[x];
    if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, WV_STATUS_COUNTS);
}

}  // namespace

namespace {

// dst[i] = src[i] for `bytes` bytes, src in pinned host memory (read by the
// device directly); 16-byte pieces, then the tail
__global__ void upload_k(uint8_t* __restrict__ dst, const uint8_t* __restrict__ src, uint64_t bytes)
{
    const uint64_t n16 = bytes / 16;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        ((uint4*)dst)[i] = ((const uint4*)src)[i];
    for (uint64_t i = n16 * 16 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t wv_upload(void* dst, const void* pinned, uint64_t bytes, hipStream_t s)
{
    if (!bytes) return hipSuccess;
    if (((uintptr_t)dst | (uintptr_t)pinned) & 15u) return hipErrorInvalidValue;
    void* src = nullptr;
    hipError_t e = hipHostGetDevicePointer(&src, const_cast<void*>(pinned), 0);
    if (e != hipSuccess) return e;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(wv_cdiv(bytes, 16 * 256), 1), 256);
    upload_k<<<grid, 256, 0, s>>>((uint8_t*)dst, (const uint8_t*)src, bytes);
    return hipGetLastError();
}

hipError_t wv_check_counts(const uint64_t* got, const uint64_t* want, uint32_t sigma, uint8_t* image, hipStream_t s)
{
    const uint32_t grid = (uint32_t)std::min<uint64_t>(wv_cdiv(sigma, DIR_THREADS), 256);
    counts_match_k<<<std::max(grid, 1u), DIR_THREADS, 0, s>>>(got, want, sigma, (uint32_t*)(image + 36));
    return hipGetLastError();
}

// ---- directories of several levels in one launch per step ----------------------

namespace {

constexpr uint32_t SD_T = 256;                 // threads, two words each
constexpr uint32_t SD_W = 2 * SD_T;            // words per chunk (64 superblocks)

struct SpanLevels {
    uint64_t bits_off[WV_MAX_LEVELS], rank_off[WV_MAX_LEVELS], sel0_off[WV_MAX_LEVELS], sel1_off[WV_MAX_LEVELS];
    uint64_t sub_off[WV_MAX_LEVELS], nsub[WV_MAX_LEVELS];
    uint64_t n[WV_MAX_LEVELS], nsel[WV_MAX_LEVELS];   // per level (chunks past a level's end count 0)
    uint32_t l0, nl;
};

__global__ void __launch_bounds__(SD_T)
span_count_k(const uint8_t* __restrict__ image, SpanLevels a, uint32_t* __restrict__ cnt)
{
    __shared__ uint32_t part[SD_T / 64];
    const uint32_t c = blockIdx.x, l = blockIdx.y;
    const uint64_t nw = wv_cdiv(a.n[l], 64);
    const uint64_t* words = (const uint64_t*)(image + a.bits_off[l]);
    const uint64_t w0 = (uint64_t)c * SD_W + 2 * threadIdx.x;
    uint32_t o = 0;
    if (nw) {   // uniform: a level of a shaped tree can be empty
        // both loads in flight (index clamped, masked after)
        const uint64_t x0 = words[min(w0, nw - 1)], x1 = words[min(w0 + 1, nw - 1)];
        o = (w0 < nw ? (uint32_t)__popcll(x0) : 0u) + (w0 + 1 < nw ? (uint32_t)__popcll(x1) : 0u);
    }
    o = wv_wave_incl_scan(o);   // lane 63 holds the wave's sum
    if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = o;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t k = 0; k < SD_T / 64; k++) s += part[k];
        cnt[(uint64_t)c * a.nl + l] = s;
    }
}

// Positions, counts and word indices of a level fit 32 bits (n < 2^32): the
// per-word work is done in 32-bit arithmetic, widened only where a u64 entry
// is stored.
__global__ void __launch_bounds__(SD_T)
span_write_k(uint8_t* __restrict__ image, SpanLevels a, const uint64_t* __restrict__ pre, uint32_t nchunks)
{
    __shared__ uint32_t wpart[SD_T / 64];
    __shared__ alignas(16) uint32_t zex[SD_W];   // zeros of the chunk before each of its words (up to the level's end)
    __shared__ uint64_t wds[SD_W];               // the chunk's words
    const uint32_t l = blockIdx.y;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n = (uint32_t)a.n[l];
    const uint32_t nw = (uint32_t)wv_cdiv(n, 64), ns = (uint32_t)wv_cdiv(n, WV_SB_BITS);
    const uint64_t* words = (const uint64_t*)(image + a.bits_off[l]);
    uint64_t* dir = (uint64_t*)(image + a.rank_off[l]);
    uint64_t* sel0 = (uint64_t*)(image + a.sel0_off[l]);
    uint64_t* sel1 = (uint64_t*)(image + a.sel1_off[l]);
    uint32_t* sub = (uint32_t*)(image + a.sub_off[l]);
    const uint32_t nsub = (uint32_t)a.nsub[l];
    // my two words of chunk c (16-byte aligned: the first is even)
    auto load2 = [&](uint32_t c, uint64_t& y0, uint64_t& y1) {
        const uint32_t w = c * SD_W + 2 * threadIdx.x;
        y0 = y1 = 0;
        if (w + 1 < nw) {
            const ulonglong2 v = *(const ulonglong2*)(words + w);
            y0 = v.x;
            y1 = v.y;
        } else if (w < nw) {
            y0 = words[w];
        }
    };
    uint64_t nx0 = 0, nx1 = 0;
    if (blockIdx.x * 4 < nchunks) load2(blockIdx.x * 4, nx0, nx1);
    for (uint32_t gi = 0; gi < 4; gi++) {   // four chunks per workgroup
        const uint32_t c = blockIdx.x * 4 + gi;
        if (c >= nchunks) break;   // uniform
        // this chunk's words were loaded one chunk ahead; load the next now
        const uint64_t x0 = nx0, x1 = nx1;
        if (gi + 1 < 4 && c + 1 < nchunks) load2(c + 1, nx0, nx1);
        const uint32_t cw = c * SD_W;
        const uint32_t cbits = (uint32_t)min<uint64_t>(64ull * cw, n);
        const uint32_t nloc = min(n - cbits, 64u * SD_W);                 // level bits in the chunk
        const uint32_t obase = (uint32_t)pre[(uint64_t)c * a.nl + l];     // ones before the chunk
        const uint32_t zbase = cbits - obase;                             // zeros before the chunk
        const uint32_t wl = 2 * threadIdx.x;                              // my first word, chunk-local
        const uint32_t o0 = __popcll(x0), o1 = __popcll(x1);
        // exclusive prefix of ones over the words of the chunk
        const uint32_t inc = wv_wave_incl_scan(o0 + o1);
        if (lane == 63) wpart[wave] = inc;
        __syncthreads();
        uint32_t off = 0, ones = 0;
        for (uint32_t k = 0; k < SD_T / 64; k++) {
            if (k < wave) off += wpart[k];
            ones += wpart[k];
        }
        const uint32_t ob0 = off + inc - (o0 + o1), ob1 = ob0 + o0;   // ones before my words
        const uint32_t z0 = min(64u * wl, nloc) - ob0, z1 = min(64u * (wl + 1), nloc) - ob1;
        zex[wl] = z0;
        zex[wl + 1] = z1;
        wds[wl] = x0;
        wds[wl + 1] = x1;
        __syncthreads();
        // sampled select: the ones / zeros of ordinal 512k in the chunk (a
        // sub-sample each, a sample when 4096 divides the ordinal)
        wv_chunk_samples(wds, zex, (uint32_t)min<uint64_t>(SD_W, nw - cw), nloc, cw, obase, zbase, ones, sub, nsub,
                      sel0, sel1);
        // one thread per superblock of the chunk: zeros before it, and the
        // zeros before each of its words 1..7 relative to that (9 bits each)
        if (threadIdx.x < SD_W / 8) {
            const uint32_t k = cw / 8 + threadIdx.x;
            if (k < ns) {
                const uint4 za = *(const uint4*)(zex + 8 * threadIdx.x), zb4 = *(const uint4*)(zex + 8 * threadIdx.x + 4);
                const uint32_t zb = za.x;
                const uint32_t lo = (za.y - zb) | ((za.z - zb) << 9) | ((za.w - zb) << 18);
                const uint32_t hi = (zb4.x - zb) | ((zb4.y - zb) << 9) | ((zb4.z - zb) << 18);
                const uint64_t blk = (uint64_t)lo | ((uint64_t)hi << 27) | ((uint64_t)(zb4.w - zb) << 54);
                *(ulonglong2*)(dir + 2 * (uint64_t)k) = make_ulonglong2((uint64_t)(zbase + zb), blk);   // 16-byte aligned
            }
        }
        __syncthreads();   // wpart and zex are rewritten by the next chunk
    }
}

__global__ void __launch_bounds__(SD_T)
span_finish_k(uint8_t* __restrict__ image, SpanLevels a, const uint64_t* __restrict__ totals)
{
    const uint32_t l = blockIdx.x;
    const uint64_t n = a.n[l], ns = wv_cdiv(n, WV_SB_BITS);
    const uint64_t ones = totals[l], zeros = n - ones;
    uint64_t* dir = (uint64_t*)(image + a.rank_off[l]);
    uint64_t* sel0 = (uint64_t*)(image + a.sel0_off[l]);
    uint64_t* sel1 = (uint64_t*)(image + a.sel1_off[l]);
    if (threadIdx.x == 0) {
        dir[2 * ns] = zeros;
        dir[2 * ns + 1] = 0;
        uint64_t* desc = (uint64_t*)(image + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * (a.l0 + l));
        desc[1] = zeros;
        desc[2] = ones;
    }
    for (uint64_t k = wv_cdiv(ones, WV_SEL_STRIDE) + threadIdx.x; k < a.nsel[l]; k += SD_T) sel1[k] = n;
    for (uint64_t k = wv_cdiv(zeros, WV_SEL_STRIDE) + threadIdx.x; k < a.nsel[l]; k += SD_T) sel0[k] = n;
    uint32_t* sub = (uint32_t*)(image + a.sub_off[l]);
    const uint64_t sub_hi = a.nsub[l] - wv_cdiv(zeros, WV_SUB_STRIDE);
    for (uint64_t k = wv_cdiv(ones, WV_SUB_STRIDE) + threadIdx.x; k < sub_hi; k += SD_T) sub[k] = (uint32_t)n;
}

}  // namespace

wv_span_dir wv_span_dir_sizes(uint64_t n, uint32_t nl)
{
    wv_span_dir z{};
    z.nl = nl;
    z.nchunks = wv_cdiv(wv_cdiv(n, 64), SD_W);
    const uint64_t items = std::max<uint64_t>(z.nchunks * nl, 1);
    uint64_t off = 0;
    z.off_cnt = off;
    off = wv_round256(off + items * 4);
    z.off_pre = off;
    off = wv_round256(off + items * 8);
    z.off_part = off;
    off = wv_round256(off + 8 * wv_scan_partials(z.nchunks, nl));
    z.off_tot = off;
    off = wv_round256(off + 8 * (uint64_t)std::max<uint32_t>(nl, 1));
    z.bytes = off;
    return z;
}

hipError_t wv_span_directory(uint8_t* image, const wv_layout_out& lay, uint32_t l0, uint32_t nl,
                             uint8_t* scratch, const wv_span_dir& sz, hipStream_t s, bool prof)
{
    if (!nl) return hipSuccess;
    SpanLevels a{};
    a.l0 = l0;
    a.nl = nl;
    for (uint32_t l = 0; l < nl; l++) {
        a.n[l] = lay.lv[l0 + l].n;
        a.nsel[l] = lay.lv[l0 + l].nsel;
        a.bits_off[l] = lay.lv[l0 + l].bits_off;
        a.rank_off[l] = lay.lv[l0 + l].rank_off;
        a.sel0_off[l] = lay.lv[l0 + l].sel0_off;
        a.sel1_off[l] = lay.lv[l0 + l].sel1_off;
        a.sub_off[l] = lay.lv[l0 + l].sub_off;
        a.nsub[l] = lay.lv[l0 + l].nsub;
    }
    uint32_t* cnt = (uint32_t*)(scratch + sz.off_cnt);
    uint64_t* pre = (uint64_t*)(scratch + sz.off_pre);
    uint64_t* tot = (uint64_t*)(scratch + sz.off_tot);
    const dim3 grid((uint32_t)sz.nchunks, nl);
    if (sz.nchunks) WV_TIMED(prof, s, "dir_count", (span_count_k<<<grid, SD_T, 0, s>>>(image, a, cnt)));
    hipError_t e = hipSuccess;
    WV_TIMED(prof, s, "dir_scan",
             e = wv_scan_u32(cnt, pre, sz.nchunks, nl, (uint64_t*)(scratch + sz.off_part), tot, s));
    if (e != hipSuccess) return e;
    if (sz.nchunks) WV_TIMED(prof, s, "dir_write", (span_write_k<<<dim3((uint32_t)wv_cdiv(sz.nchunks, 4), nl), SD_T, 0, s>>>(image, a, pre, (uint32_t)sz.nchunks)));
    WV_TIMED(prof, s, "dir_finish", (span_finish_k<<<nl, SD_T, 0, s>>>(image, a, tot)));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    WV_TIMED(prof, s, "dir_explicit", e = launch_xsel(image, lay.lv + l0, nl, s));
    return e;
}
