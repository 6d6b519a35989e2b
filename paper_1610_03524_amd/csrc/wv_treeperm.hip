// wv_treeperm.hip -- tree levels from wavelet-matrix levels.
//
// Level l of the balanced tree (Sec. 2) and level l of the wavelet matrix
// (Sec. 4.3) hold the same runs: one run per group of symbols that share
// their top l key bits, holding bit l of those symbols in input order.  The
// tree lays the runs out in the numeric order of the groups, the matrix in
// the order of the groups' bit-reversed prefixes (every matrix level is a
// stable partition by the previous bit).  A tree level is therefore the
// matrix level with its runs moved, and the matrix is what the multi-level
// passes build fastest.
//
// A shaped tree (Sec. 4.3) is handled the same way over codewords padded at
// the bottom to the longest code length h: a symbol whose code ends above
// level l is a leaf there; its padded prefix cannot be the prefix of another
// codeword (the code is prefix-free), so the groups of leaves are separate
// runs, which the tree level simply leaves out.
//
// A deep shaped tree whose long codes are rare is gathered from two matrices:
// the levels above the split from a matrix over the top bits of every
// codeword, the deeper ones from a matrix over the long-code symbols alone
// (only they reach those levels, each group of them in input order).
//
// A multiary tree (Sec. 4.3) with D-bit digits keeps the binary levels bD:
// its level b holds the same runs as matrix level bD, with each symbol's
// digit (its bits on matrix levels bD .. bD+D-1) in place of one bit.
//
// The host derives, from the symbol counts, every kept run's bit offset on
// the matrix level and on the tree level, and the first run of every 256-word
// tile of the tree levels; one thread per output word gathers its bits from
// the runs that cover it, and for a multiary tree the same launch counts the
// digits of every counter range (Sec. 5's rank counters).
#include <algorithm>
#include <vector>

#include "wv_treeperm.h"

namespace {

// Split shaped build.  A block takes KB symbols; with 16-byte aligned input
// every thread reads V = 16 / sizeof(T) consecutive symbols per row with one
// load (rows of KB_T * V symbols), else (and in a ragged last block) one
// symbol per thread per row.
constexpr uint32_t KB_T = 256, KB = 4096;

template <typename T>
struct SymVec {
    static constexpr uint32_t V = 16 / sizeof(T);
    T v[V];
};

// symbols [i, i + V) of the block's row (`vec`: one 16-byte load)
template <typename T>
__device__ inline void load_syms(const T* __restrict__ S, uint64_t i, uint64_t n, bool vec, SymVec<T>& out)
{
    constexpr uint32_t V = SymVec<T>::V;
    if (vec) {
        const uint4 q = *(const uint4*)(S + i);
        __builtin_memcpy(out.v, &q, 16);
    } else {
#pragma unroll
        for (uint32_t k = 0; k < V; k++) out.v[k] = i + k < n ? S[i + k] : (T)0;
    }
}

// The split table of a symbol: its top h1 code bits, bit 16 set when its code
// is longer than h1 (0 for symbols without a code).  Staged in LDS when sigma
// is small; the workgroups then loop over the blocks of KB symbols.
constexpr uint32_t KTAB_LDS = 8192;
constexpr uint32_t KB_GRID = 1280;   // five resident workgroups per CU

__device__ inline const uint32_t* stage_table(const uint32_t* __restrict__ ktab, uint32_t sigma, uint32_t* lds)
{
    if (sigma > KTAB_LDS) return ktab;
    for (uint32_t x = threadIdx.x; x < sigma; x += KB_T) lds[x] = ktab[x];
    __syncthreads();
    return lds;
}

// Padded codeword keys, keys[i] = ktab[S[i]] (0 for a symbol >= sigma, which
// the validation has flagged): the table in LDS when sigma is small, blocks
// of KB symbols read and written in 16-byte pieces.
template <typename T>
__global__ void __launch_bounds__(KB_T)
tree_keys_k(const T* __restrict__ S, uint64_t n, uint32_t sigma, const uint32_t* __restrict__ ktab,
            uint32_t* __restrict__ keys, uint64_t nblocks)
{
    constexpr uint32_t V = SymVec<T>::V, ROWS = KB / (KB_T * V);
    __shared__ uint32_t tab_s[KTAB_LDS];
    const uint32_t* tab = stage_table(ktab, sigma, tab_s);
    for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const uint64_t b0 = blk * KB;
        const bool vec = (((uintptr_t)S & 15u) == 0) && (((uintptr_t)keys & 15u) == 0) && b0 + KB <= n;
        SymVec<T> sv[ROWS];
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) load_syms(S, b0 + (r * KB_T + threadIdx.x) * V, n, vec, sv[r]);
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) {
            const uint64_t i0 = b0 + (r * KB_T + threadIdx.x) * V;
            uint32_t kk[V];
#pragma unroll
            for (uint32_t k = 0; k < V; k++) {
                const uint32_t x = (uint32_t)sv[r].v[k];
                kk[k] = i0 + k < n && x < sigma ? tab[x] : 0u;
            }
            if (vec) {
#pragma unroll
                for (uint32_t k = 0; k < V; k += 4) *(uint4*)(keys + i0 + k) = make_uint4(kk[k], kk[k + 1], kk[k + 2], kk[k + 3]);
            } else {
#pragma unroll
                for (uint32_t k = 0; k < V; k++)
                    if (i0 + k < n) keys[i0 + k] = kk[k];
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(KB_T)
tree_keys_split_k(const T* __restrict__ S, uint64_t n, uint32_t sigma, const uint32_t* __restrict__ ktab,
                  uint16_t* __restrict__ keys, uint32_t* __restrict__ bcnt, uint16_t* __restrict__ lmask,
                  uint64_t nblocks)
{
    constexpr uint32_t V = SymVec<T>::V, ROWS = KB / (KB_T * V);
    __shared__ uint32_t tab_s[KTAB_LDS];
    __shared__ uint32_t wc[KB_T / 64];
    const uint32_t* tab = stage_table(ktab, sigma, tab_s);
    for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const uint64_t b0 = blk * KB;
        const bool vec = (((uintptr_t)S & 15u) == 0) && b0 + KB <= n;
        SymVec<T> sv[ROWS];
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) load_syms(S, b0 + (r * KB_T + threadIdx.x) * V, n, vec, sv[r]);
        uint32_t c = 0;
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) {
            const uint64_t i0 = b0 + (r * KB_T + threadIdx.x) * V;
            uint16_t kk[V];
            uint32_t m = 0;   // bit k: symbol k of the thread's row piece has a long code
#pragma unroll
            for (uint32_t k = 0; k < V; k++) {
                const uint32_t x = (uint32_t)sv[r].v[k];
                const uint32_t t = i0 + k < n && x < sigma ? tab[x] : 0u;
                kk[k] = (uint16_t)t;
                c += t >> 16;
                m |= (t >> 16) << k;
            }
            lmask[(blk * ROWS + r) * KB_T + threadIdx.x] = (uint16_t)m;
            if (vec) {
                // V 16-bit keys: 32 bytes (8-bit symbols), 16 (16-bit) or 8 (32-bit)
                if constexpr (V >= 8) {
#pragma unroll
                    for (uint32_t k = 0; k < V; k += 8) {
                        uint4 q;
                        __builtin_memcpy(&q, kk + k, 16);
                        *(uint4*)(keys + i0 + k) = q;
                    }
                } else {
                    uint2 q;
                    __builtin_memcpy(&q, kk, 8);
                    *(uint2*)(keys + i0) = q;
                }
            } else {
#pragma unroll
                for (uint32_t k = 0; k < V; k++)
                    if (i0 + k < n) keys[i0 + k] = kk[k];
            }
        }
        c = wv_wave_incl_scan(c);
        if ((threadIdx.x & 63) == 63) wc[threadIdx.x >> 6] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (uint32_t w = 0; w < KB_T / 64; w++) t += wc[w];
            bcnt[blk] = t;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(KB_T)
tree_long_keys_k(const T* __restrict__ S, uint64_t n, const uint32_t* __restrict__ codes,
                 const uint32_t* __restrict__ lens, uint32_t h, const uint64_t* __restrict__ boff,
                 const uint16_t* __restrict__ lmask, uint32_t* __restrict__ lkeys, uint64_t nlong, uint64_t nblocks)
{
    constexpr uint32_t V = SymVec<T>::V, ROWS = KB / (KB_T * V);
    __shared__ uint32_t wsum[ROWS][KB_T / 64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (uint64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
        const uint64_t b0 = blk * KB;
        // long symbols per thread and row, as the key kernel marked them
        // (S is read again only at those positions); symbols are in input
        // order row by row, thread by thread inside a row
        uint32_t lm[ROWS], inc[ROWS];   // lm: bit k = symbol k of the thread's row piece is long
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) {
            lm[r] = lmask[(blk * ROWS + r) * KB_T + threadIdx.x];
            inc[r] = wv_wave_incl_scan((uint32_t)__popc(lm[r]));
            if (lane == 63) wsum[r][wave] = inc[r];
        }
        __syncthreads();
        uint64_t base = boff[blk];
#pragma unroll
        for (uint32_t r = 0; r < ROWS; r++) {
            uint64_t rank = base + inc[r] - (uint32_t)__popc(lm[r]);
            for (uint32_t w = 0; w < wave; w++) rank += wsum[r][w];
            if (lm[r]) {
                const uint64_t i0 = b0 + (r * KB_T + threadIdx.x) * V;
#pragma unroll
                for (uint32_t k = 0; k < V; k++) {
                    if (!((lm[r] >> k) & 1u)) continue;
                    const uint32_t x = (uint32_t)S[i0 + k];   // marked only below n and sigma
                    if (rank < nlong) lkeys[rank] = codes[x] << (h - lens[x]);
                    rank++;
                }
            }
            for (uint32_t w = 0; w < KB_T / 64; w++) base += wsum[r][w];
        }
        __syncthreads();
    }
}

// `nb` (1..64) bits of a level bit string starting at bit `pos`; the array
// has one readable word past its last word
__device__ inline uint64_t bits_at(const uint64_t* __restrict__ w, uint64_t pos, uint32_t nb)
{
    const uint64_t i = pos >> 6;
    const uint32_t o = (uint32_t)(pos & 63);
    uint64_t v = w[i] >> o;
    if (o && o + nb > 64) v |= w[i + 1] << (64 - o);
    return nb >= 64 ? v : (v & ((1ull << nb) - 1ull));
}

struct PermArgs {
    const wv_perm_level* lv;
    const wv_perm_seg* seg;
    const uint32_t* tile_seg;
    uint32_t tile0[WV_MAX_LEVELS + 1];
    uint32_t nlev;
    wv_perm_counts cnt;
};

// One thread per output word, a workgroup per tile of one level: the run
// holding the word's first bit is searched among the runs that cover the tile
// (from the tile's first run to the next tile's), then its bits are gathered
// run by run.  COUNT (multiary levels): each wave is one 64-word range of one
// level, and its scans of the per-word digit counts give the range totals and
// the counts before every 8-word sub-range (Sec. 5's two-level counters,
// taken here instead of in a second pass over the level).
template <bool COUNT>
__global__ void __launch_bounds__(WV_PERM_TILE)
perm_runs_k(PermArgs a)
{
    const uint32_t b = blockIdx.x;
    uint32_t l = 0;
    while (l + 1 < a.nlev && a.tile0[l + 1] <= b) l++;   // uniform
    const wv_perm_level L = a.lv[l];
    const uint64_t w = (uint64_t)(b - a.tile0[l]) * WV_PERM_TILE + threadIdx.x;
    const uint64_t nw = wv_cdiv(L.nbits, 64);
    uint64_t out = 0;
    if (w < nw) {
        const uint64_t p0 = w * 64, end = min(p0 + 64, L.nbits);
        // the run holding bit p0: the last one starting at or before it
        uint64_t lo = a.tile_seg[b];
        uint64_t hi = b + 1 < a.tile0[l + 1] ? a.tile_seg[b + 1] : L.seg0 + L.nseg - 1;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) >> 1;
            if (a.seg[mid].dst <= p0) lo = mid; else hi = mid - 1;
        }
        for (uint64_t p = p0, k = lo; p < end; k++) {
            const wv_perm_seg g = a.seg[k];
            const uint64_t in = p - g.dst;
            const uint32_t take = (uint32_t)min(end - p, g.len - in);
            out |= bits_at(L.src, g.src + in, take) << (p - p0);
            p += take;
        }
        L.dst[w] = out;
    }
    if (COUNT) {
        const wv_perm_counts& cnt = a.cnt;
        const uint32_t lane = threadIdx.x & 63, D = cnt.D, P = wv_digits_per_word(D), d = 1u << D;
        const uint64_t m = L.nbits >> (D >> 1);   // the level's digits (D = 1, 2, 4)
        const uint64_t r = w >> 6, sk = w >> 3;
        if (r >= wv_mranges(m, D)) return;   // whole waves
        const uint32_t c = w < nw ? (uint32_t)min<uint64_t>(P, m - w * P) : 0u;
        const bool subw = (lane & 7) == 0 && sk < wv_msubs(m, D);
        for (uint32_t g0 = 0; g0 < d; g0 += 4) {
            uint64_t pack = 0;   // up to four 16-bit sub-range counters
            for (uint32_t gg = 0; gg < 4 && g0 + gg < d; gg++) {
                const uint32_t v = wv_count_digit(out, D, g0 + gg, c);
                const uint32_t inc = wv_wave_incl_scan(v);
                if (lane == 63) cnt.rng_cnt[(r * cnt.M + l) * d + g0 + gg] = inc;
                pack |= (uint64_t)(inc - v) << (16 * gg);
            }
            if (subw) {
                if (d == 2) *(uint32_t*)(L.sub + sk * d) = (uint32_t)pack;
                else *(uint64_t*)(L.sub + sk * d + g0) = pack;
            }
        }
    }
}

// ---- balanced trees: runs from the symbol counts, on the device ----------------

__device__ inline uint32_t brev_bits(uint32_t v, uint32_t nbits) { return nbits ? (__brev(v) >> (32 - nbits)) : 0u; }

// the symbol counts as 32-bit values over the whole key space (0 past sigma)
__global__ void group_counts_k(const uint64_t* __restrict__ counts, uint32_t sigma, uint32_t keys,
                               uint32_t* __restrict__ cnt)
{
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < keys; x += gridDim.x * blockDim.x)
        cnt[x] = x < sigma ? (uint32_t)counts[x] : 0u;
}

// V[2^l - 1 + r] = symbols under the prefix brev(r) on level l, for l < K
__global__ void group_levels_k(const uint64_t* __restrict__ C, uint32_t K, uint32_t* __restrict__ V)
{
    const uint32_t total = (1u << K) - 1u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint32_t l = 31 - __clz(i + 1);
        const uint32_t g = brev_bits(i + 1 - (1u << l), l);
        const uint32_t sh = K - l;
        V[i] = (uint32_t)(C[(uint64_t)(g + 1) << sh] - C[(uint64_t)g << sh]);
    }
}

struct GroupArgs {
    wv_group_level lv[WV_MAX_LEVELS];
    uint32_t tile0[WV_MAX_LEVELS + 1];
    uint32_t nlev, K, D;
    const uint64_t* C;
    const uint64_t* P;
    wv_perm_counts cnt;
};

// One thread per output word, a workgroup per 256-word tile of one level: the
// group holding each run of the word is found by a binary search in C (the
// last prefix starting at or before the symbol), its place in the matrix
// order read from P, and its bits gathered.  COUNT as in perm_runs_k.
template <bool COUNT>
__global__ void __launch_bounds__(WV_PERM_TILE)
perm_groups_k(GroupArgs a)
{
    const uint32_t b = blockIdx.x;
    uint32_t t = 0;
    while (t + 1 < a.nlev && a.tile0[t + 1] <= b) t++;   // uniform
    const wv_group_level L = a.lv[t];
    const uint64_t w = (uint64_t)(b - a.tile0[t]) * WV_PERM_TILE + threadIdx.x;
    const uint64_t nw = wv_cdiv(L.nbits, 64);
    const uint32_t D = a.D, dsh = D == 1 ? 0u : (D == 2 ? 1u : 2u);
    uint64_t out = 0;
    if (w < nw) {
        const uint64_t p0 = w * 64, end = min(p0 + 64, L.nbits);
        const uint32_t l = L.l, sh = a.K - l;
        const uint32_t G = 1u << l, base = G - 1u;
        const uint64_t pbase = a.P[base];
        for (uint64_t p = p0; p < end;) {
            const uint64_t q = p >> dsh;   // symbol position
            uint32_t lo = 0, hi = G - 1u;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1u) >> 1;
                if (a.C[(uint64_t)mid << sh] <= q) lo = mid; else hi = mid - 1u;
            }
            const uint64_t start = a.C[(uint64_t)lo << sh], stop = a.C[(uint64_t)(lo + 1) << sh];
            if (stop <= q) break;   // counts short of the level (a symbol >= sigma): the rest stays 0
            const uint64_t src = a.P[base + brev_bits(lo, l)] - pbase;
            const uint64_t in = p - (start << dsh);
            const uint32_t take = (uint32_t)min(end - p, ((stop - start) << dsh) - in);
            out |= bits_at(L.src, (src << dsh) + in, take) << (p - p0);
            p += take;
        }
        L.dst[w] = out;
    }
    if (COUNT) {
        const wv_perm_counts& cnt = a.cnt;
        const uint32_t lane = threadIdx.x & 63, P = wv_digits_per_word(D), d = 1u << D;
        const uint64_t r = w >> 6, sk = w >> 3;
        if (r >= wv_mranges(cnt.m, D)) return;   // whole waves
        const uint32_t c = w < nw ? (uint32_t)min<uint64_t>(P, cnt.m - w * P) : 0u;
        const bool subw = (lane & 7) == 0 && sk < wv_msubs(cnt.m, D);
        for (uint32_t g0 = 0; g0 < d; g0 += 4) {
            uint64_t pack = 0;   // up to four 16-bit sub-range counters
            for (uint32_t gg = 0; gg < 4 && g0 + gg < d; gg++) {
                const uint32_t v = wv_count_digit(out, D, g0 + gg, c);
                const uint32_t inc = wv_wave_incl_scan(v);
                if (lane == 63) cnt.rng_cnt[(r * cnt.M + t) * d + g0 + gg] = inc;
                pack |= (uint64_t)(inc - v) << (16 * gg);
            }
            if (subw) {
                if (d == 2) *(uint32_t*)(L.sub + sk * d) = (uint32_t)pack;
                else *(uint64_t*)(L.sub + sk * d + g0) = pack;
            }
        }
    }
}

// the low 64/D bits of x moved to bit positions 0, D, 2D, ... (D = 1, 2, 4)
__device__ inline uint64_t spread(uint64_t x, uint32_t D)
{
    if (D == 2) {
        x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
        x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
        x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
        x = (x | (x << 2)) & 0x3333333333333333ull;
        x = (x | (x << 1)) & 0x5555555555555555ull;
    } else if (D == 4) {
        x = (x | (x << 24)) & 0x000000FF000000FFull;
        x = (x | (x << 12)) & 0x000F000F000F000Full;
        x = (x | (x << 6)) & 0x0303030303030303ull;
        x = (x | (x << 3)) & 0x1111111111111111ull;
    }
    return x;
}

// Digits of one multiary level, in the order of matrix level bD: the symbol
// at position i there has its digit's D bits on matrix levels bD .. bD+D-1,
// each level's position found from the previous one by the matrix map (a
// zero moves to its rank among zeros, a one to Z + its rank among ones).
// A wave takes DW consecutive words of level bD (64 positions each, padding
// bits 0): one rank query per word and the zeros below each lane give every
// position's place on the next level; the loads of the DW words are issued
// together.  The 64 digits of a word fill D words of the digit string (digit
// e at bits D*e .. D*e+D-1, low bit first).
constexpr uint32_t DW = 8;

template <uint32_t D>
__global__ void __launch_bounds__(256)
digits_k(wv_digit_set set, uint64_t n, uint64_t nwords)
{
    const wv_digit_levels& a = set.lv[blockIdx.y];   // digit level t = blockIdx.y
    uint64_t* __restrict__ out = set.out[blockIdx.y];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t nw0 = wv_cdiv(n, 64);
    const uint64_t bw = wave * DW;
    if (bw >= nw0) return;   // whole waves: the ballots below need every lane
    uint64_t w0[DW], rb[DW];
#pragma unroll
    for (uint32_t j = 0; j < DW; j++) w0[j] = bw + j < nw0 ? a.words[0][bw + j] : 0ull;
    uint32_t d[DW];
#pragma unroll
    for (uint32_t j = 0; j < DW; j++) d[j] = (uint32_t)(w0[j] >> lane) & 1u;
    if (D > 1) {
#pragma unroll
        for (uint32_t j = 0; j < DW; j++) rb[j] = bw + j < nw0 ? wv_rank0(a.words[0], a.dir[0], (bw + j) * 64) : 0ull;
        const uint64_t Z0 = wv_rank0(a.words[0], a.dir[0], n);
        // positions past n follow position 0 (their digits are masked below),
        // so every lane loads and the loads of the DW words go out together
        uint64_t p[DW];
#pragma unroll
        for (uint32_t j = 0; j < DW; j++) {
            const uint64_t i = (bw + j) * 64 + lane;
            const uint64_t r0 = rb[j] + __builtin_amdgcn_mbcnt_hi((uint32_t)(~w0[j] >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)~w0[j], 0u));
            p[j] = i < n ? (d[j] ? Z0 + (i - r0) : r0) : 0ull;
        }
#pragma unroll
        for (uint32_t k = 1; k < D; k++) {
            const uint64_t Zk = k + 1 < D ? wv_rank0(a.words[k], a.dir[k], n) : 0ull;
#pragma unroll
            for (uint32_t j = 0; j < DW; j++) {
                const uint32_t bit = (uint32_t)(a.words[k][p[j] >> 6] >> (p[j] & 63)) & 1u;
                d[j] = (d[j] << 1) | bit;
                if (k + 1 < D) {
                    const uint64_t rk = wv_rank0(a.words[k], a.dir[k], p[j]);
                    p[j] = bit ? Zk + (p[j] - rk) : rk;
                }
            }
        }
    }
    const uint32_t per = 64 / D;
    const uint64_t pmask = per == 64 ? ~0ull : ((1ull << per) - 1ull);
#pragma unroll
    for (uint32_t j = 0; j < DW; j++) {
        if (bw + j >= nw0) break;   // uniform
        const uint32_t dj = (bw + j) * 64 + lane < n ? d[j] : 0u;
        uint64_t bt[D];
#pragma unroll
        for (uint32_t t = 0; t < D; t++) bt[t] = __ballot((dj >> t) & 1u);
        if (lane < D) {
            uint64_t w = 0;
#pragma unroll
            for (uint32_t t = 0; t < D; t++) w |= spread((bt[t] >> (lane * per)) & pmask, D) << t;
            const uint64_t wi = (bw + j) * D + lane;
            if (wi < nwords) out[wi] = w;
        }
    }
}

// The low popcount(m) bits of x, in order, moved to the set positions of m
// (bit expand, the inverse of compress; the parallel-suffix network of
// Hacker's Delight, Sec. 7-5): six masks from m, then six shift-and-merge steps.
__device__ inline uint64_t expand64(uint64_t x, uint64_t m)
{
    const uint64_t m0 = m;
    uint64_t mk = ~m << 1;   // a one where the next lower bit is a zero of m
    uint64_t mv[6];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        // parallel suffix: bit b of mp = parity of the zeros of m below b
        uint64_t mp = mk ^ (mk << 1);
        mp ^= mp << 2;
        mp ^= mp << 4;
        mp ^= mp << 8;
        mp ^= mp << 16;
        mp ^= mp << 32;
        mv[i] = mp & m;                               // bits that move by 2^i
        m = (m ^ mv[i]) | (mv[i] >> (1 << i));
        mk &= ~mp;
    }
#pragma unroll
    for (int i = 5; i >= 0; i--) {
        const uint64_t t = x << (1 << i);
        x = (x & ~mv[i]) | (t & mv[i]);
    }
    return x & m0;
}

// 64 bits of a level from bit `pos` (pos < n); the word after the last is not
// read (bits past n are never used)
__device__ inline uint64_t bits64(const uint64_t* __restrict__ w, uint64_t pos, uint64_t nw)
{
    const uint64_t i = pos >> 6;
    const uint32_t o = (uint32_t)(pos & 63);
    const uint64_t lo = w[i], hi = w[min(i + 1, nw - 1)];
    return o ? (lo >> o) | (hi << (64 - o)) : lo;
}

// The same for 2-bit digits, one thread per word of level bD and no rank
// query per word: the zeros of word k go, in order, to consecutive positions
// of level bD+1 from zr (the zeros before the word), its ones to consecutive
// positions from Z + (64k - zr).  The low digit bits of the word are therefore
// the 64 bits of level bD+1 at zr expanded onto its zeros, merged with the 64
// bits at Z + 64k - zr expanded onto its ones.  A workgroup scans its words'
// zero counts; the zeros before its first word and Z come from a scan of the
// zero counts of every workgroup (digit_zeros_k).
constexpr uint32_t DG = 256;

__global__ void __launch_bounds__(DG)
digits2_k(wv_digit_set set, uint64_t n, uint64_t nwords, const uint64_t* __restrict__ zpre,
          const uint64_t* __restrict__ ztot, uint32_t T)
{
    const uint32_t t = blockIdx.y;   // digit level
    const wv_digit_levels& a = set.lv[t];
    uint64_t* __restrict__ out = set.out[t];
    __shared__ uint32_t wsum[DG / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t nw0 = wv_cdiv(n, 64);
    const uint64_t c0 = (uint64_t)blockIdx.x * DG;
    const uint64_t k = c0 + tid;
    const uint64_t r0c = zpre[(uint64_t)blockIdx.x * T + t];   // zeros of level 2t before the block
    const uint64_t Z0 = ztot[t];
    const uint64_t w = k < nw0 ? a.words[0][k] : 0ull;
    const uint32_t valid = k < nw0 ? (uint32_t)min<uint64_t>(64, n - k * 64) : 0u;
    const uint64_t vm = valid >= 64 ? ~0ull : ((1ull << valid) - 1ull);
    const uint32_t z = valid - (uint32_t)__popcll(w);   // padding bits are 0
    const uint32_t inc = wv_wave_incl_scan(z);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (k >= nw0) return;
    uint32_t off = 0;
    for (uint32_t q = 0; q < wave; q++) off += wsum[q];
    const uint64_t zr = r0c + off + inc - z;   // zeros of level bD before word k
    const uint64_t A = bits64(a.words[1], min(zr, n - 1), nw0);
    const uint64_t B = bits64(a.words[1], min(Z0 + (k * 64 - zr), n - 1), nw0);
    const uint64_t lo = expand64(A, ~w & vm) | expand64(B, w);
    // digit e of the word at bits 2e (level bD+1) and 2e+1 (level bD)
    out[2 * k] = spread(lo & 0xFFFFFFFFull, 2) | (spread(w & 0xFFFFFFFFull, 2) << 1);
    if (2 * k + 1 < nwords) out[2 * k + 1] = spread(lo >> 32, 2) | (spread(w >> 32, 2) << 1);
}

// One group of a level: the symbols [a, b) of the key-sorted symbol list
// sharing the level's key prefix (live: on the tree level), or a block of
// symbols whose codes have ended (dead: left out of the level, padded with
// zeros below their code)
struct Group {
    uint32_t a, b;
    uint64_t count;
    bool live;
};

}  // namespace

void wv_tree_segments(const std::vector<uint64_t>& counts, uint32_t key_bits, const uint32_t* codes,
                      const uint32_t* lens, std::vector<wv_perm_seg>& segs, std::vector<uint64_t>& seg0)
{
    // (padded key, symbols, code length) of every symbol present, by key
    struct Sym { uint64_t key, count; uint32_t len; };
    std::vector<Sym> sy;
    for (uint64_t x = 0; x < counts.size(); x++) {
        if (!counts[x]) continue;
        if (codes) sy.push_back(Sym{(uint64_t)codes[x] << (key_bits - lens[x]), counts[x], lens[x]});
        else sy.push_back(Sym{x, counts[x], key_bits});
    }
    std::sort(sy.begin(), sy.end(), [](const Sym& a, const Sym& b) { return a.key < b.key; });
    const uint32_t ns = (uint32_t)sy.size();
    std::vector<uint64_t> pre(ns + 1, 0);
    for (uint32_t i = 0; i < ns; i++) pre[i + 1] = pre[i] + sy[i].count;
    segs.clear();
    seg0.assign(key_bits + 1, 0);
    if (!ns) return;
    // a group with one symbol whose code ends at or above level l is dead
    auto make = [&](uint32_t a, uint32_t b, uint32_t l) {
        return Group{a, b, pre[b] - pre[a], !(b - a == 1 && sy[a].len <= l)};
    };
    // Level l of the matrix orders the groups by their bit-reversed prefix,
    // which is the order of level l-1 stably partitioned by key bit l-1: the
    // zero children of every group in that order, then the one children.
    // A dead symbol's padding bits are zeros, so dead symbols next to each
    // other stay next to each other and are kept as one block.
    std::vector<Group> morder{make(0, ns, 0)}, zeros, ones;   // matrix order
    std::vector<Group> num, nnum;                              // live groups by key
    if (morder[0].live) num.push_back(morder[0]);
    std::vector<uint64_t> src_at(ns, 0);
    auto push = [](std::vector<Group>& v, const Group& g) {
        if (!g.live && !v.empty() && !v.back().live) v.back().count += g.count;
        else v.push_back(g);
    };
    for (uint32_t l = 0; l < key_bits; l++) {
        seg0[l] = segs.size();
        uint64_t acc = 0;
        for (const Group& g : morder) {
            if (g.live) src_at[g.a] = acc;
            acc += g.count;
        }
        uint64_t dst = 0;
        for (const Group& g : num) {
            segs.push_back(wv_perm_seg{dst, src_at[g.a], g.count});
            dst += g.count;
        }
        if (l + 1 == key_bits) break;
        // split every live group by key bit l (counted from the top)
        const uint32_t sh = key_bits - 1 - l;
        auto split = [&](const Group& g) {
            return (uint32_t)(std::partition_point(sy.begin() + g.a, sy.begin() + g.b,
                                                   [&](const Sym& y) { return !((y.key >> sh) & 1u); }) - sy.begin());
        };
        zeros.clear();
        ones.clear();
        for (const Group& g : morder) {
            if (!g.live) {
                push(zeros, g);
                continue;
            }
            const uint32_t m = split(g);
            if (m > g.a) push(zeros, make(g.a, m, l + 1));
            if (m < g.b) push(ones, make(m, g.b, l + 1));
        }
        morder.swap(zeros);
        for (const Group& g : ones) push(morder, g);
        nnum.clear();
        for (const Group& g : num) {
            const uint32_t m = split(g);
            if (m > g.a) {
                const Group c = make(g.a, m, l + 1);
                if (c.live) nnum.push_back(c);
            }
            if (m < g.b) {
                const Group c = make(m, g.b, l + 1);
                if (c.live) nnum.push_back(c);
            }
        }
        num.swap(nnum);
    }
    seg0[key_bits] = segs.size();
}

hipError_t wv_tree_keys(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma, const uint32_t* ktab,
                        uint32_t* keys, hipStream_t s)
{
    if (!n) return hipSuccess;
    const uint64_t nb = wv_tree_key_blocks(n);
    const uint32_t g = (uint32_t)std::min<uint64_t>(nb, KB_GRID);
    if (sym_bytes == 1) tree_keys_k<uint8_t><<<g, KB_T, 0, s>>>((const uint8_t*)S, n, sigma, ktab, keys, nb);
    else if (sym_bytes == 2) tree_keys_k<uint16_t><<<g, KB_T, 0, s>>>((const uint16_t*)S, n, sigma, ktab, keys, nb);
    else tree_keys_k<uint32_t><<<g, KB_T, 0, s>>>((const uint32_t*)S, n, sigma, ktab, keys, nb);
    return hipGetLastError();
}

void wv_key_table(const uint32_t* codes, const uint32_t* lens, uint32_t sigma, uint32_t h, std::vector<uint32_t>& tab)
{
    tab.assign(sigma, 0u);
    for (uint32_t x = 0; x < sigma; x++)
        if (lens[x]) tab[x] = codes[x] << (h - lens[x]);
}

namespace {

// zeros of every DG-word block of the levels 2t (t < T), column t of row b
__global__ void __launch_bounds__(DG)
digit_zeros_k(wv_digit_words a, uint64_t n, uint32_t T, uint32_t* __restrict__ cnt)
{
    __shared__ uint32_t wsum[DG / 64];
    const uint32_t t = blockIdx.y;
    const uint64_t nw0 = wv_cdiv(n, 64);
    const uint64_t k = (uint64_t)blockIdx.x * DG + threadIdx.x;
    uint32_t z = 0;
    if (k < nw0) z = (uint32_t)min<uint64_t>(64, n - k * 64) - (uint32_t)__popcll(a.w[t][k]);   // padding bits are 0
    z = wv_wave_incl_scan(z);
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = z;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < DG / 64; w++) s += wsum[w];
        cnt[(uint64_t)blockIdx.x * T + t] = s;
    }
}

}  // namespace

uint64_t wv_tree_key_blocks(uint64_t n) { return wv_cdiv(n ? n : 1, KB); }

uint64_t wv_digit_blocks(uint64_t n) { return wv_cdiv(wv_cdiv(n ? n : 1, 64), DG); }

hipError_t wv_digit_zero_counts(const wv_digit_words& a, uint64_t n, uint32_t T, uint32_t* cnt, hipStream_t s)
{
    if (!n || !T) return hipSuccess;
    digit_zeros_k<<<dim3((uint32_t)wv_digit_blocks(n), T), DG, 0, s>>>(a, n, T, cnt);
    return hipGetLastError();
}

void wv_split_table(const uint32_t* codes, const uint32_t* lens, uint32_t sigma, uint32_t h, uint32_t h1,
                    std::vector<uint32_t>& tab)
{
    tab.assign(sigma, 0u);
    for (uint32_t x = 0; x < sigma; x++)
        if (lens[x]) tab[x] = ((codes[x] << (h - lens[x])) >> (h - h1)) | (lens[x] > h1 ? WV_SPLIT_LONG : 0u);
}

hipError_t wv_tree_keys_split(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma, const uint32_t* ktab,
                              uint16_t* keys, uint32_t* bcnt, uint16_t* lmask, hipStream_t s)
{
    if (!n) return hipSuccess;
    const uint64_t nb = wv_tree_key_blocks(n);
    const uint32_t g = (uint32_t)std::min<uint64_t>(nb, KB_GRID);
    if (sym_bytes == 1)
        tree_keys_split_k<uint8_t><<<g, KB_T, 0, s>>>((const uint8_t*)S, n, sigma, ktab, keys, bcnt, lmask, nb);
    else if (sym_bytes == 2)
        tree_keys_split_k<uint16_t><<<g, KB_T, 0, s>>>((const uint16_t*)S, n, sigma, ktab, keys, bcnt, lmask, nb);
    else
        tree_keys_split_k<uint32_t><<<g, KB_T, 0, s>>>((const uint32_t*)S, n, sigma, ktab, keys, bcnt, lmask, nb);
    return hipGetLastError();
}

uint64_t wv_tree_lmask_bytes(uint64_t n, uint32_t sym_bytes)
{
    // ROWS = sym_bytes rows of KB_T threads per block, a 16-bit mask each
    return wv_tree_key_blocks(n) * sym_bytes * KB_T * 2;
}

hipError_t wv_tree_long_keys(const void* S, uint64_t n, uint32_t sym_bytes, const uint32_t* codes, const uint32_t* lens,
                             uint32_t h, const uint64_t* boff, const uint16_t* lmask, uint32_t* lkeys, uint64_t nlong,
                             hipStream_t s)
{
    if (!n || !nlong) return hipSuccess;
    const uint64_t nb = wv_tree_key_blocks(n);
    const uint32_t g = (uint32_t)std::min<uint64_t>(nb, KB_GRID);
    if (sym_bytes == 1)
        tree_long_keys_k<uint8_t><<<g, KB_T, 0, s>>>((const uint8_t*)S, n, codes, lens, h, boff, lmask, lkeys, nlong, nb);
    else if (sym_bytes == 2)
        tree_long_keys_k<uint16_t><<<g, KB_T, 0, s>>>((const uint16_t*)S, n, codes, lens, h, boff, lmask, lkeys, nlong, nb);
    else
        tree_long_keys_k<uint32_t><<<g, KB_T, 0, s>>>((const uint32_t*)S, n, codes, lens, h, boff, lmask, lkeys, nlong, nb);
    return hipGetLastError();
}

hipError_t wv_tree_digits(const wv_digit_set& a, uint32_t T, uint64_t n, uint32_t D, const uint64_t* zpre,
                          const uint64_t* ztot, hipStream_t s)
{
    if (!n || !T) return hipSuccess;
    if (T > WV_MAX_LEVELS) return hipErrorInvalidValue;
    const uint32_t g = (uint32_t)wv_cdiv(wv_cdiv(wv_cdiv(n, 64), DW), 4);   // 4 waves per block
    const uint64_t nw = wv_cdiv(n * D, 64);
    if (D == 1) digits_k<1><<<dim3(g, T), 256, 0, s>>>(a, n, nw);
    else if (D == 2) digits2_k<<<dim3((uint32_t)wv_digit_blocks(n), T), DG, 0, s>>>(a, n, nw, zpre, ztot, T);
    else if (D == 4) digits_k<4><<<dim3(g, T), 256, 0, s>>>(a, n, nw);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

uint32_t wv_tree_tiles(const std::vector<wv_perm_level>& lv, const std::vector<wv_perm_seg>& segs, bool counting,
                       std::vector<uint32_t>& tile0, std::vector<uint32_t>& tile_seg)
{
    tile0.assign(lv.size() + 1, 0);
    tile_seg.clear();
    for (uint32_t l = 0; l < lv.size(); l++) {
        const wv_perm_level& L = lv[l];
        tile0[l] = (uint32_t)tile_seg.size();
        const uint64_t words = counting ? wv_cdiv(wv_cdiv(L.nbits, 64), 64) * 64 : wv_cdiv(L.nbits, 64);
        if (!L.nseg) continue;   // no bits, no tiles
        const uint64_t tiles = wv_cdiv(words, WV_PERM_TILE), last = L.seg0 + L.nseg - 1;
        uint64_t k = L.seg0;
        for (uint64_t t = 0; t < tiles; t++) {
            const uint64_t p = t * WV_PERM_TILE * 64;
            while (k < last && segs[k + 1].dst <= p) k++;
            tile_seg.push_back((uint32_t)k);
        }
    }
    tile0[lv.size()] = (uint32_t)tile_seg.size();
    return tile0[lv.size()];
}

wv_group_ws wv_group_ws_sizes(uint32_t K)
{
    wv_group_ws z{};
    const uint64_t keys = 1ull << K;
    uint64_t off = 0;
    auto bump = [&](uint64_t bytes) { const uint64_t at = off; off = wv_round256(off + bytes); return at; };
    z.off_cnt = bump(keys * 4);
    z.off_C = bump((keys + 1) * 8);
    z.off_V = bump(keys * 4);
    z.off_P = bump(keys * 8);
    z.off_part = bump(8 * wv_scan_partials(keys, 1));
    z.off_tot = bump(8);
    z.bytes = off;
    return z;
}

hipError_t wv_tree_group_runs(const uint64_t* counts, uint32_t sigma, uint32_t K, uint8_t* ws,
                              const wv_group_ws& z, hipStream_t s)
{
    if (K > WV_GROUP_MAX_BITS) return hipErrorInvalidValue;
    const uint32_t keys = 1u << K;
    uint32_t* cnt = (uint32_t*)(ws + z.off_cnt);
    uint64_t* C = (uint64_t*)(ws + z.off_C);
    uint32_t* V = (uint32_t*)(ws + z.off_V);
    uint64_t* P = (uint64_t*)(ws + z.off_P);
    uint64_t* part = (uint64_t*)(ws + z.off_part);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(wv_cdiv(keys, 256), 1024);
    group_counts_k<<<grid, 256, 0, s>>>(counts, sigma, keys, cnt);
    hipError_t e = wv_scan_u32(cnt, C, keys, 1, part, C + keys, s);   // C[keys] = symbols counted
    if (e != hipSuccess) return e;
    if (keys > 1) {
        group_levels_k<<<grid, 256, 0, s>>>(C, K, V);
        e = wv_scan_u32(V, P, keys - 1, 1, part, (uint64_t*)(ws + z.off_tot), s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t wv_tree_permute_groups(const wv_group_level* lv, uint32_t nlev, uint32_t K, uint32_t D, const uint8_t* ws,
                                  const wv_group_ws& z, const wv_perm_counts* counts, hipStream_t s)
{
    if (!nlev || nlev > WV_MAX_LEVELS) return nlev ? hipErrorInvalidValue : hipSuccess;
    if (D != 1 && D != 2 && D != 4) return hipErrorInvalidValue;
    GroupArgs a{};
    uint32_t tiles = 0;
    for (uint32_t t = 0; t < nlev; t++) {
        a.lv[t] = lv[t];
        a.tile0[t] = tiles;
        const uint64_t nw = wv_cdiv(lv[t].nbits, 64);
        const uint64_t words = counts ? wv_cdiv(nw, 64) * 64 : nw;
        if (lv[t].nbits) tiles += (uint32_t)wv_cdiv(words, WV_PERM_TILE);
    }
    a.tile0[nlev] = tiles;
    a.nlev = nlev;
    a.K = K;
    a.D = D;
    a.C = (const uint64_t*)(ws + z.off_C);
    a.P = (const uint64_t*)(ws + z.off_P);
    if (!tiles) return hipSuccess;
    if (counts) {
        a.cnt = *counts;
        perm_groups_k<true><<<tiles, WV_PERM_TILE, 0, s>>>(a);
    } else {
        perm_groups_k<false><<<tiles, WV_PERM_TILE, 0, s>>>(a);
    }
    return hipGetLastError();
}

hipError_t wv_tree_permute(const wv_perm_level* lv_dev, uint32_t nlev, const wv_perm_seg* seg_dev,
                           const uint32_t* tile_seg_dev, const uint32_t* tile0, const wv_perm_counts* counts,
                           hipStream_t s)
{
    if (!nlev || nlev > WV_MAX_LEVELS) return nlev ? hipErrorInvalidValue : hipSuccess;
    const uint32_t tiles = tile0[nlev];
    if (!tiles) return hipSuccess;
    PermArgs a{};
    a.lv = lv_dev;
    a.seg = seg_dev;
    a.tile_seg = tile_seg_dev;
    for (uint32_t l = 0; l <= nlev; l++) a.tile0[l] = tile0[l];
    a.nlev = nlev;
    if (counts) {
        if (counts->D != 1 && counts->D != 2 && counts->D != 4) return hipErrorInvalidValue;
        a.cnt = *counts;
        perm_runs_k<true><<<tiles, WV_PERM_TILE, 0, s>>>(a);
    } else {
        perm_runs_k<false><<<tiles, WV_PERM_TILE, 0, s>>>(a);
    }
    return hipGetLastError();
}
