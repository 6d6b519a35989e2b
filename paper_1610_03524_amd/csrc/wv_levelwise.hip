// wv_levelwise.hip -- one-level-per-pass builder for every kind.
//
// This is the direct form of the definitions (Sec. 2 for the balanced tree,
// Sec. 4.3 for the wavelet matrix, shaped and multiary trees): level l is
// emitted from the symbols in the order of level l, its directory is built,
// and every symbol is then moved to its place on level l+1:
//   wavelet matrix:  0-bits to rank0(i), 1-bits to Z_l + rank1(i);
//   trees:           inside its node, to the start of its child plus its
//                    rank among the node's symbols with the same bit/digit.
// Tree nodes are described by a node table built on the host from the
// symbol counts (node start, child starts, child ids); symbols carry their
// node id from level to level.  The wavelet-matrix builds use the faster
// multi-level partition passes of wv_wm_passes.hip; this path serves the
// trees and the one-level-per-pass matrix variant.
#include "wv_internal.h"
#include "wv_levelwise.h"

namespace {

constexpr int EMIT_THREADS = 512;   // one 512-bit superblock per block
constexpr int LW_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(EMIT_THREADS)
emit_bits_k(const void* __restrict__ keys, uint64_t m, wv_keyfn f, uint64_t* __restrict__ words,
            uint32_t* __restrict__ sb_ones)
{
    __shared__ uint32_t cnt[EMIT_THREADS / 64];
    const uint64_t i = (uint64_t)blockIdx.x * EMIT_THREADS + threadIdx.x;
    uint32_t b = 0;
    if (i < m) b = wv_digit(f, wv_load_sym<T>(keys, i));
    const uint64_t w = __ballot(b);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        const uint64_t wi = i >> 6;
        if (wi < wv_cdiv(m, 64)) words[wi] = w;
        cnt[wave] = __popcll(w);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < EMIT_THREADS / 64; k++) s += cnt[k];
        sb_ones[blockIdx.x] = s;
    }
}

template <typename T>
__global__ void __launch_bounds__(LW_THREADS)
emit_digits_k(const void* __restrict__ keys, uint64_t m, wv_keyfn f, uint64_t* __restrict__ words)
{
    const uint64_t w = (uint64_t)blockIdx.x * LW_THREADS + threadIdx.x;
    const uint32_t P = 64u / f.D;
    if (w >= wv_cdiv(m, P)) return;
    uint64_t word = 0;
    for (uint32_t t = 0; t < P; t++) {
        const uint64_t i = w * P + t;
        if (i < m) word |= (uint64_t)wv_digit(f, wv_load_sym<T>(keys, i)) << (t * f.D);
    }
    words[w] = word;
}

template <typename T>
__global__ void __launch_bounds__(LW_THREADS)
scatter_wm_k(const void* __restrict__ keys, uint64_t m, wv_keyfn f, const uint64_t* __restrict__ words,
             const uint64_t* __restrict__ dir, const uint64_t* __restrict__ zl, uint32_t* __restrict__ out)
{
    const uint64_t i = (uint64_t)blockIdx.x * LW_THREADS + threadIdx.x;
    if (i >= m) return;
    const uint32_t key = wv_load_sym<T>(keys, i);
    const uint32_t b = wv_digit(f, key);
    const uint64_t r0 = wv_rank0(words, dir, i);
    const uint64_t dst = b ? (*zl + (i - r0)) : r0;
    out[dst] = key;
}

template <typename T>
__global__ void __launch_bounds__(LW_THREADS)
scatter_tree_k(const void* __restrict__ keys, const uint32_t* __restrict__ nodes_in, uint64_t m, wv_keyfn f,
               const uint64_t* __restrict__ words, const uint64_t* __restrict__ dir, wv_node_table nt,
               uint32_t* __restrict__ keys_out, uint32_t* __restrict__ nodes_out)
{
    const uint64_t i = (uint64_t)blockIdx.x * LW_THREADS + threadIdx.x;
    if (i >= m) return;
    const uint32_t key = wv_load_sym<T>(keys, i);
    const uint32_t b = wv_digit(f, key);
    const uint32_t k = nodes_in ? nodes_in[i] : 0u;
    const uint64_t s = nt.start[k];
    const uint64_t zi = wv_rank0(words, dir, i), zs = wv_rank0(words, dir, s);
    const uint64_t rel = b ? ((i - s) - (zi - zs)) : (zi - zs);
    const uint32_t c = nt.child[2 * k + b];
    if (c & WV_LEAF) return;   // the symbol reached its leaf (or no child)
    const uint64_t dst = nt.child_start[2 * k + b] + rel;
    keys_out[dst] = key;
    nodes_out[dst] = c;
}

template <typename T>
__global__ void __launch_bounds__(LW_THREADS)
scatter_multi_k(const void* __restrict__ keys, const uint32_t* __restrict__ nodes_in, uint64_t m, wv_keyfn f,
                const uint64_t* __restrict__ words, const uint8_t* __restrict__ cnt, wv_node_table nt,
                uint32_t* __restrict__ keys_out, uint32_t* __restrict__ nodes_out)
{
    const uint64_t i = (uint64_t)blockIdx.x * LW_THREADS + threadIdx.x;
    if (i >= m) return;
    const uint32_t D = f.D, d = 1u << D;
    const uint32_t key = wv_load_sym<T>(keys, i);
    const uint32_t g = wv_digit(f, key);
    const uint32_t k = nodes_in ? nodes_in[i] : 0u;
    const uint64_t s = nt.start[k];
    const uint64_t rel = wv_mrank(words, cnt, m, D, g, i) - wv_mrank(words, cnt, m, D, g, s);
    const uint32_t c = nt.child[(uint64_t)k * d + g];
    if (c & WV_LEAF) return;
    const uint64_t dst = nt.child_start[(uint64_t)k * d + g] + rel;
    keys_out[dst] = key;
    nodes_out[dst] = c;
}

inline uint32_t blocks_for(uint64_t items, uint32_t threads) { return (uint32_t)wv_cdiv(items, threads); }

template <typename T>
hipError_t emit_level(const void* keys, uint64_t m, const wv_keyfn& f, uint8_t* image, const wv_level& L,
                      uint32_t* sb_ones, hipStream_t s)
{
    if (!m) return hipSuccess;
    uint64_t* words = (uint64_t*)(image + L.bits_off);
    if (f.D == 1 && f.mode != WV_KEY_DIGIT_MULTI)
        emit_bits_k<T><<<blocks_for(m, EMIT_THREADS), EMIT_THREADS, 0, s>>>(keys, m, f, words, sb_ones);
    else
        emit_digits_k<T><<<blocks_for(wv_cdiv(m, 64u / f.D), LW_THREADS), LW_THREADS, 0, s>>>(keys, m, f, words);
    return hipGetLastError();
}

template <typename T>
hipError_t scatter_level(const void* keys, const uint32_t* nodes_in, uint64_t m, const wv_keyfn& f,
                         const uint8_t* image, const wv_level& L, const uint64_t* zl, const wv_node_table& nt,
                         int kind, uint32_t* keys_out, uint32_t* nodes_out, hipStream_t s)
{
    if (!m) return hipSuccess;
    const uint64_t* words = (const uint64_t*)(image + L.bits_off);
    const uint32_t g = blocks_for(m, LW_THREADS);
    if (kind != WT_KIND_WM && f.D >= 2)   // digit levels: multiary and shaped multiary trees
        scatter_multi_k<T><<<g, LW_THREADS, 0, s>>>(keys, nodes_in, m, f, words, image + L.rank_off, nt,
                                                     keys_out, nodes_out);
    else if (kind == WT_KIND_WM)
        scatter_wm_k<T><<<g, LW_THREADS, 0, s>>>(keys, m, f, words, (const uint64_t*)(image + L.rank_off), zl, keys_out);
    else if (kind == WT_KIND_MULTIARY)
        scatter_multi_k<T><<<g, LW_THREADS, 0, s>>>(keys, nodes_in, m, f, words, image + L.rank_off, nt,
                                                     keys_out, nodes_out);
    else
        scatter_tree_k<T><<<g, LW_THREADS, 0, s>>>(keys, nodes_in, m, f, words,
                                                    (const uint64_t*)(image + L.rank_off), nt, keys_out, nodes_out);
    return hipGetLastError();
}

template <typename T>
hipError_t run_levels(const wv_lw_args& a, hipStream_t s)
{
    const int kind = a.kind;
    const wv_layout_out& lay = *a.lay;
    const void* keys = a.S;
    const uint32_t* nodes_in = nullptr;
    uint32_t* kbuf[2] = {a.keys_a, a.keys_b};
    uint32_t* nbuf[2] = {a.nodes_a, a.nodes_b};
    int cur = 0;
    bool first = true;
    hipError_t e;
    for (uint32_t l = 0; l < a.nlevels; l++) {
        const wv_level& L = lay.lv[l];
        const uint64_t m = L.n;
        wv_keyfn f = a.keyfn(l);
        WV_TIMED(a.profile, s, "lw_emit",
                 e = first ? emit_level<T>(keys, m, f, a.image, L, a.dir.sb_ones, s)
                           : emit_level<uint32_t>(keys, m, f, a.image, L, a.dir.sb_ones, s));
        if (e != hipSuccess) return e;
        WV_TIMED(a.profile, s, "lw_directory",
                 e = wv_multi_levels(kind, a.arity_log2) ? wv_multiary_counters(a.image, &L, 1, f.D, a.mdir, s)
                                                         : wv_binary_directory(a.image, l, L, a.dir, a.zl, s));
        if (e != hipSuccess) return e;
        if (l + 1 == a.nlevels) break;
        WV_TIMED(a.profile, s, "lw_scatter",
                 e = first ? scatter_level<T>(keys, nodes_in, m, f, a.image, L, a.zl, a.nt, kind, kbuf[cur],
                                              nbuf[cur], s)
                           : scatter_level<uint32_t>(keys, nodes_in, m, f, a.image, L, a.zl, a.nt, kind, kbuf[cur],
                                                     nbuf[cur], s));
        if (e != hipSuccess) return e;
        keys = kbuf[cur];
        nodes_in = kind == WT_KIND_WM ? nullptr : nbuf[cur];
        cur ^= 1;
        first = false;
    }
    return hipSuccess;
}

}  // namespace

wv_keyfn wv_lw_args::keyfn(uint32_t l) const
{
    wv_keyfn f{};
    f.D = kind == WT_KIND_MULTIARY ? arity_log2 : 1u;
    if (kind == WT_KIND_SHAPED) {
        f.mode = WV_KEY_CODE;
        f.D = arity_log2 >= 2 ? arity_log2 : 1u;
        f.level = l;
        f.codes = codes;
        f.lens = lens;
    } else {
        f.mode = kind == WT_KIND_MULTIARY ? WV_KEY_DIGIT_MULTI : WV_KEY_SYMBOL;
        f.shift = key_bits - f.D * (l + 1);
    }
    return f;
}

hipError_t wv_run_levelwise(const wv_lw_args& a, uint32_t sym_bytes, hipStream_t s)
{
    if (sym_bytes == 1) return run_levels<uint8_t>(a, s);
    if (sym_bytes == 2) return run_levels<uint16_t>(a, s);
    return run_levels<uint32_t>(a, s);
}
