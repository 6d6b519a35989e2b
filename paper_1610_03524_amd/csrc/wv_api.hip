// wv_api.hip -- C-ABI entry points of libwavelet (declared in wavelet.h).
//
// Planning (image layout and workspace), the host-side pieces of the tree
// builds (node tables from symbol counts, canonical Huffman codewords) and
// the dispatch to the device passes.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "wv_internal.h"
#include "wv_levelwise.h"
#include "wv_treeperm.h"
#include "wv_wm_passes.h"

bool wv_trace_on()
{
    static const bool on = [] {
        const char* v = std::getenv("WT_TRACE");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    return on;
}

void wv_trace(const char* fmt, ...)
{
    char line[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(line, sizeof line, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[wt] %s\n", line);
}

namespace {

struct Plan {
    int kind = 0;
    uint32_t sigma = 0, sym_bytes = 0, D = 1, key_bits = 0, nlevels = 0, tau = 0;
    uint64_t n = 0, nnodes_image = 0, ncoded = 0;
    bool levelwise = false;
    wv_layout_in lin{};
    wv_layout_out lay{};
    // workspace regions (byte offsets)
    uint64_t ws_scalars = 0, ws_keys_a = 0, ws_keys_b = 0, ws_nodes_a = 0, ws_nodes_b = 0;
    uint64_t ws_sb_ones = 0, ws_sb_pre = 0, ws_partial = 0, ws_counts = 0, ws_mtot = 0;
    uint64_t ws_nt_start = 0, ws_nt_cstart = 0, ws_nt_child = 0, node_bound = 0;
    uint64_t ws_codes = 0, ws_lens = 0, ws_wm = 0;
    // trees gathered from matrix levels (balanced and shaped binary trees)
    bool from_matrix = false;
    uint64_t ws_tkeys = 0, ws_tmp = 0, tmp_stride = 0, ws_segs = 0, seg_bound = 0, tile_bound = 0;
    uint64_t ws_tmpimg = 0, ws_digits = 0, dstride = 0;   // multiary: matrix image, digit strings
    wv_layout_out tlay{};
    uint64_t ws_timgb = 0;     // split shaped trees over digits: the image of matrix B
    wv_layout_out tlayb{};
    // shaped trees split at level h1: matrix A over the top h1 bits of every
    // codeword (p.wm), matrix B over the whole codewords of the nlong symbols
    // whose codes are longer than h1 (wmb)
    uint32_t h1 = 0;
    uint64_t nlong = 0, ws_lkeys = 0, ws_btmp = 0, btmp_stride = 0, ws_wmb = 0;
    uint64_t ws_bcnt = 0, ws_boff = 0, ws_bpart = 0, nkblocks = 0, ws_sdir = 0, ws_ktab = 0;   // ws_sdir: directory scratch, all levels
    uint64_t ws_lmask = 0;     // long-code marks of the split key kernel
    wv_wm_plan wmb{};
    // balanced trees of at most 8 key bits built in one pass straight into
    // tree order (domain decomposition), no matrix levels in between
    bool direct_tree = false;
    // balanced binary and multiary trees: runs derived on the device
    bool dev_runs = false;
    wv_group_ws gz{};
    uint64_t ws_group = 0;
    uint64_t ws_scounts = 0;   // shaped trees: the shape's counts, checked on the device
    uint64_t ws_bytes = 0;
    wv_wm_plan wm{};
};

bool is_tree(int kind) { return kind == WT_KIND_WT || kind == WT_KIND_SHAPED || kind == WT_KIND_MULTIARY; }

uint64_t bump(uint64_t& off, uint64_t bytes)
{
    uint64_t at = off;
    off = wv_round256(off + bytes);
    return at;
}

// The coded symbols of a shape, ordered by codeword padded at the bottom to
// the longest code length h (D-bit digits; D = 1 for binary codes).  In that
// order a codeword shares its top lcp digits with its predecessor and adds
// len - 1 - lcp new proper prefixes (tree nodes), and the code is
// prefix-free iff no codeword's top len digits equal its successor's.
struct Coded {
    uint64_t key;
    uint32_t len, sym;
};

int sorted_codes(const wt_shape& sh, uint32_t sigma, uint32_t h, std::vector<Coded>& cs, uint64_t* nnodes,
                 uint32_t D = 1)
{
    cs.clear();
    for (uint32_t x = 0; x < sigma; x++)
        if (sh.code_len[x])
            cs.push_back(Coded{(uint64_t)sh.codes[x] << (D * (h - sh.code_len[x])), sh.code_len[x], x});
    std::sort(cs.begin(), cs.end(), [](const Coded& a, const Coded& b) { return a.key < b.key; });
    uint64_t nodes = 0;
    for (size_t i = 0; i < cs.size(); i++) {
        uint32_t lcp = 0;
        if (i) {
            const uint64_t x = cs[i - 1].key ^ cs[i].key;
            lcp = x ? ((uint32_t)__builtin_clzll(x) - (64 - D * h)) / D : h;
            if (lcp >= std::min(cs[i - 1].len, cs[i].len)) return WT_EINVAL;   // one code is a prefix of the other
            nodes += cs[i].len - 1 - lcp;
        } else {
            nodes += cs[i].len;
        }
    }
    *nnodes = nodes;
    return WT_OK;
}

// workspace of the gather's level descriptors, runs and tile table
inline uint64_t seg_bytes(uint64_t segs, uint64_t tiles)
{
    return wv_round256(WV_MAX_LEVELS * sizeof(wv_perm_level)) + wv_round256(segs * sizeof(wv_perm_seg)) + tiles * 4 + 256;
}

int make_plan_impl(int kind, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
                   const wt_tuning* tune, Plan& p)
{
    if (kind < WT_KIND_WT || kind > WT_KIND_MULTIARY) return WT_EINVAL;
    if (sigma == 0) return WT_EINVAL;
    if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4) return WT_EINVAL;
    if (n >= (1ull << 32)) return WT_EUNSUP;
    p.kind = kind;
    p.n = n;
    p.sigma = sigma;
    p.sym_bytes = sym_bytes;
    const uint32_t L = wv_key_bits(sigma);
    p.levelwise = tune && ((tune->flags & WT_FLAG_LEVELWISE) || tune->tau == 1);
    if (kind == WT_KIND_WM && shape && shape->codes) return WT_EINVAL;

    std::vector<uint64_t> level_n;
    if (kind == WT_KIND_WT || kind == WT_KIND_WM) {
        p.D = 1;
        p.key_bits = L;
        p.nlevels = L;
        level_n.assign(L, n);
    } else if (kind == WT_KIND_MULTIARY) {
        if (!shape || shape->arity_log2 < 1 || shape->arity_log2 > 4) return WT_EINVAL;
        p.D = shape->arity_log2;
        p.nlevels = (L + p.D - 1) / p.D;
        p.key_bits = p.D * p.nlevels;
        level_n.assign(p.nlevels, n);
    } else {
        if (!shape || !shape->codes || !shape->code_len || !shape->counts) return WT_EINVAL;
        // codewords of D-bit digits (arity_log2 0 or 1: binary), lengths in
        // digits, at most 32 bits per codeword
        if (shape->arity_log2 > 4) return WT_EINVAL;
        p.D = std::max(shape->arity_log2, 1u);
        uint32_t h = 0;
        uint64_t total = 0;
        for (uint32_t s = 0; s < sigma; s++) {
            const uint32_t len = shape->code_len[s];
            if ((uint64_t)len * p.D > 32) return WT_EUNSUP;
            if (len && (shape->codes[s] >> (len * p.D))) return WT_EINVAL;
            if (len) p.ncoded++;
            h = std::max(h, len);
            total += shape->counts[s];
            if (shape->counts[s] && !len) return WT_ERANGE;
        }
        if (h == 0 || total != n) return WT_EINVAL;
        p.key_bits = h * p.D;
        p.nlevels = h;
        // 3-bit digits do not pack words exactly: level by level
        if (p.D == 3) p.levelwise = true;
        level_n.assign(h, 0);
        for (uint32_t s = 0; s < sigma; s++)
            for (uint32_t l = 0; l < shape->code_len[s]; l++) level_n[l] += shape->counts[s];
    }
    if (p.nlevels > WV_MAX_LEVELS) return WT_EUNSUP;

    // image layout
    p.lin = wv_layout_in{};
    p.lin.kind = (uint32_t)kind;
    p.lin.arity_log2 = wv_multi_levels(kind, p.D) ? p.D : 1u;
    p.lin.nlevels = p.nlevels;
    p.lin.key_bits = p.key_bits;
    p.lin.sigma = sigma;
    p.lin.n = n;
    p.lin.ncoded = p.ncoded;
    for (uint32_t l = 0; l < p.nlevels; l++) p.lin.level_n[l] = level_n[l];
    if (kind == WT_KIND_SHAPED) {
        // internal nodes: distinct proper prefixes of the codewords
        std::vector<Coded> cs;
        const int rc = sorted_codes(*shape, sigma, p.nlevels, cs, &p.nnodes_image, p.D);
        if (rc) return rc;
        p.lin.nnodes = p.nnodes_image;
    }
    wv_layout(p.lin, p.lay);

    // node-table bound for the tree builds
    if (kind == WT_KIND_SHAPED) {
        p.node_bound = std::max<uint64_t>(p.nnodes_image, 1);
    } else if (is_tree(kind)) {
        uint64_t b = 0;
        for (uint32_t be = 0; be < p.nlevels; be++) {
            const uint32_t sh = p.key_bits - p.D * be;
            uint64_t a = sh >= 64 ? 1 : (((uint64_t)(sigma - 1) >> sh) + 1);
            uint64_t full = (p.D * be >= 40) ? ~0ull : (1ull << (p.D * be));
            b += std::min(std::min(a, full), std::max<uint64_t>(n, 1));
        }
        p.node_bound = b;
    }

    // workspace
    const uint32_t d = 1u << p.D;
    const uint64_t ns = wv_cdiv(n, WV_SB_BITS);
    const bool multi = wv_multi_levels(kind, p.D);
    const uint64_t nr = multi ? wv_mranges(n, p.D) : 0;
    // multiary counters are built for all levels at once: M * d columns
    const uint64_t mcols = multi ? (uint64_t)d * p.nlevels : 0;
    const uint64_t dir_items = std::max<uint64_t>(std::max(ns, nr * mcols), 1);
    uint64_t off = 0;
    p.ws_scalars = bump(off, 256);
    p.ws_sb_ones = bump(off, dir_items * 4);
    p.ws_sb_pre = bump(off, dir_items * 8);
    p.ws_partial = bump(off, 8 * std::max(wv_scan_partials(ns, 1), wv_scan_partials(nr, (uint32_t)mcols)));
    p.ws_mtot = bump(off, 8 * std::max<uint64_t>(mcols, 1));
    if (kind == WT_KIND_WM && !p.levelwise) {
        int rc = wv_wm_make_plan(n, sigma, sym_bytes, tune, p.wm);
        if (rc) return rc;
        p.levelwise = !p.wm.enabled;
    }
    // Balanced trees whose key bits one pass covers (sigma <= 256): the
    // domain decomposition of Sec. 4.2.  The chunks of the pass are the K
    // sub-sequences; each chunk's run of a node goes to the node's start in
    // tree order plus the node's symbols in the chunks before it (prefix sums
    // over the per-chunk counts), the words two chunks share are OR-ed.  The
    // levels are written straight into the image.
    if (kind == WT_KIND_WT && !p.levelwise && n && L <= 8) {
        wv_wm_plan a{};
        if (wv_wm_make_plan(n, sigma, sym_bytes, tune, a) == WT_OK && a.enabled && a.tau == a.L) {
            a.tree_order = true;
            p.direct_tree = true;
            p.wm = a;
            p.tau = a.tau;
            p.ws_wm = bump(off, a.ws_bytes);
            p.ws_bytes = off;
            return WT_OK;
        }
    }
    // balanced and shaped trees: matrix passes over the (padded) keys, then
    // the runs of every level moved to tree order (levels of digits of 1, 2
    // or 4 bits, which pack words exactly, assembled from the matrix levels
    // first)
    if ((kind == WT_KIND_WT || ((kind == WT_KIND_SHAPED || kind == WT_KIND_MULTIARY) && p.D != 3)) &&
        !p.levelwise && n && p.key_bits <= 31) {
        const uint32_t sig_k = kind == WT_KIND_WT ? sigma : (1u << p.key_bits);
        const uint32_t sb_k = kind == WT_KIND_SHAPED ? 4u : sym_bytes;
        p.from_matrix = wv_wm_make_plan(n, sig_k, sb_k, tune, p.wm) == WT_OK && p.wm.enabled &&
                        p.wm.L == p.key_bits;
    }
    if (p.from_matrix && multi && kind == WT_KIND_SHAPED && p.key_bits > WV_SPLIT_BITS) {
        // as for binary codewords: when codewords longer than WV_SPLIT_BITS
        // bits are rare, matrix A takes the top WV_SPLIT_BITS bits of every
        // padded codeword (16-bit keys, fewer passes) and matrix B the whole
        // codewords of the long-code symbols alone (WV_SPLIT_BITS is a
        // multiple of D = 2, 4: the split falls between digit levels)
        uint64_t nlong = 0;
        for (uint32_t x = 0; x < sigma; x++)
            if (shape->code_len[x] * p.D > WV_SPLIT_BITS) nlong += shape->counts[x];
        wv_wm_plan a{}, b{};
        if (nlong * WV_SPLIT_SHARE <= n && wv_wm_make_plan(n, 1u << WV_SPLIT_BITS, 2, tune, a) == WT_OK && a.enabled &&
            (!nlong || (wv_wm_make_plan(nlong, 1u << p.key_bits, 4, tune, b) == WT_OK && b.enabled))) {
            p.h1 = WV_SPLIT_BITS;
            p.nlong = nlong;
            p.wm = a;
            p.wmb = b;
        }
    }
    if (p.from_matrix && multi) {
        // digit levels (multiary trees, shaped trees over D-bit digits): the
        // matrix levels in a workspace image, then the digit strings
        p.tau = p.wm.tau;
        p.ws_wm = bump(off, p.wm.ws_bytes);
        auto matrix_layout = [&](uint64_t m, uint32_t levels, wv_layout_out& out) {
            wv_layout_in tl{};
            tl.kind = WT_KIND_WM;
            tl.arity_log2 = 1;
            tl.nlevels = levels;
            tl.key_bits = levels;
            tl.sigma = sigma;
            tl.n = m;
            for (uint32_t l = 0; l < levels; l++) tl.level_n[l] = m;
            wv_layout(tl, out);
        };
        matrix_layout(n, p.h1 ? p.h1 : p.key_bits, p.tlay);
        p.ws_tmpimg = bump(off, p.tlay.image_bytes);
        p.dstride = wv_round256((wv_cdiv(n * p.D, 64) + 1) * 8);   // one readable word past each string
        p.ws_digits = bump(off, p.dstride * p.nlevels);
        if (p.h1) {
            // 16-bit keys of every symbol, whole codewords of the long ones
            p.ws_tkeys = bump(off, n * 2);
            p.nkblocks = wv_tree_key_blocks(n);
            p.ws_bcnt = bump(off, p.nkblocks * 4);
            p.ws_boff = bump(off, p.nkblocks * 8 + 8);
            p.ws_bpart = bump(off, 8 * wv_scan_partials(p.nkblocks, 1) + 8);
            p.ws_lmask = bump(off, wv_tree_lmask_bytes(n, sym_bytes));
            if (p.nlong) {
                p.ws_wmb = bump(off, p.wmb.ws_bytes);
                matrix_layout(p.nlong, p.key_bits, p.tlayb);
                p.ws_timgb = bump(off, p.tlayb.image_bytes);
                p.ws_lkeys = bump(off, p.nlong * 4);
            }
        }
        if (kind == WT_KIND_SHAPED) {
            // padded codeword keys; runs from the shape's counts on the host
            if (!p.h1) p.ws_tkeys = bump(off, n * 4);
            p.seg_bound = p.nnodes_image;
            p.tile_bound = wv_tree_tile_bound(n, p.D, p.nlevels);
            p.ws_segs = bump(off, seg_bytes(p.seg_bound, p.tile_bound));
            p.ws_counts = bump(off, (uint64_t)sigma * 8);
            // codes, lengths, padded-key table and the shape's counts next
            // to each other: one upload
            p.ws_codes = bump(off, (uint64_t)sigma * 4);
            p.ws_lens = bump(off, (uint64_t)sigma * 4);
            p.ws_ktab = bump(off, (uint64_t)sigma * 4);
            p.ws_scounts = bump(off, (uint64_t)sigma * 8);
            p.ws_bytes = off;
            return WT_OK;
        }
        if (p.key_bits <= WV_GROUP_MAX_BITS) {
            p.dev_runs = true;
            p.gz = wv_group_ws_sizes(p.key_bits);
            p.ws_group = bump(off, p.gz.bytes);
        } else {
            for (uint32_t b = 0; b < p.nlevels; b++)
                p.seg_bound += std::min<uint64_t>((((uint64_t)sigma - 1) >> (p.key_bits - p.D * b)) + 1, n);
            p.tile_bound = wv_tree_tile_bound(n, p.D, p.nlevels);
            p.ws_segs = bump(off, seg_bytes(p.seg_bound, p.tile_bound));
        }
        p.ws_counts = bump(off, (uint64_t)sigma * 8);
        p.ws_bytes = off;
        return WT_OK;
    }
    if (p.from_matrix && kind == WT_KIND_SHAPED && p.D == 1 && p.key_bits > WV_SPLIT_BITS) {
        // codes longer than WV_SPLIT_BITS are rare in a skewed alphabet: the
        // first matrix then needs 16-bit keys and fewer passes, and the deep
        // levels come from a small second matrix over those symbols alone
        uint64_t nlong = 0;
        for (uint32_t x = 0; x < sigma; x++)
            if (shape->code_len[x] > WV_SPLIT_BITS) nlong += shape->counts[x];
        wv_wm_plan a{}, b{};
        if (nlong * WV_SPLIT_SHARE <= n && wv_wm_make_plan(n, 1u << WV_SPLIT_BITS, 2, tune, a) == WT_OK && a.enabled &&
            (!nlong || (wv_wm_make_plan(nlong, 1u << p.key_bits, 4, tune, b) == WT_OK && b.enabled))) {
            p.h1 = WV_SPLIT_BITS;
            p.nlong = nlong;
            p.wm = a;
            p.wmb = b;
        }
    }
    if (p.from_matrix && p.h1) {
        p.tau = p.wm.tau;
        p.ws_wm = bump(off, p.wm.ws_bytes);
        p.tmp_stride = wv_round256(wv_bits_bytes(n) + 8);   // one readable word past each level
        p.ws_tmp = bump(off, p.tmp_stride * p.h1);
        p.ws_tkeys = bump(off, n * 2);
        p.nkblocks = wv_tree_key_blocks(n);
        p.ws_bcnt = bump(off, p.nkblocks * 4);
        p.ws_boff = bump(off, p.nkblocks * 8 + 8);
        p.ws_bpart = bump(off, 8 * wv_scan_partials(p.nkblocks, 1) + 8);
        p.ws_lmask = bump(off, wv_tree_lmask_bytes(n, sym_bytes));
        if (p.nlong) {
            p.ws_wmb = bump(off, p.wmb.ws_bytes);
            p.btmp_stride = wv_round256(wv_bits_bytes(p.nlong) + 8);
            p.ws_btmp = bump(off, p.btmp_stride * p.key_bits);
            p.ws_lkeys = bump(off, p.nlong * 4);
        }
        p.seg_bound = p.nnodes_image;
        p.tile_bound = wv_tree_tile_bound(n, 1, p.key_bits);
        p.ws_segs = bump(off, seg_bytes(p.seg_bound, p.tile_bound));
        p.ws_counts = bump(off, (uint64_t)sigma * 8);
        // codes, lengths, key table and the shape's counts next to each other: one upload
        p.ws_codes = bump(off, (uint64_t)sigma * 4);
        p.ws_lens = bump(off, (uint64_t)sigma * 4);
        p.ws_ktab = bump(off, (uint64_t)sigma * 4);
        p.ws_scounts = bump(off, (uint64_t)sigma * 8);
        p.ws_sdir = bump(off, wv_span_dir_sizes(n, p.key_bits).bytes);
        p.ws_bytes = off;
        return WT_OK;
    }
    if (p.from_matrix) {
        p.tau = p.wm.tau;
        p.ws_wm = bump(off, p.wm.ws_bytes);
        p.tmp_stride = wv_round256(wv_bits_bytes(n) + 8);   // one readable word past each level
        p.ws_tmp = bump(off, p.tmp_stride * p.key_bits);
        if (kind == WT_KIND_SHAPED) p.ws_tkeys = bump(off, n * 4);
        if (kind == WT_KIND_SHAPED) {
            p.seg_bound = p.nnodes_image;
        } else if (p.key_bits <= WV_GROUP_MAX_BITS) {
            p.dev_runs = true;
            p.gz = wv_group_ws_sizes(p.key_bits);
            p.ws_group = bump(off, p.gz.bytes);
        } else {
            for (uint32_t l = 0; l < p.key_bits; l++)
                p.seg_bound += std::min<uint64_t>((((uint64_t)sigma - 1) >> (p.key_bits - l)) + 1, n);
        }
        if (!p.dev_runs) {
            p.tile_bound = wv_tree_tile_bound(n, 1, p.key_bits);
            p.ws_segs = bump(off, seg_bytes(p.seg_bound, p.tile_bound));
        }
        p.ws_counts = bump(off, (uint64_t)sigma * 8);
        if (kind == WT_KIND_SHAPED) {
            // codes, lengths, padded-key table and the shape's counts next to
            // each other: one upload
            p.ws_codes = bump(off, (uint64_t)sigma * 4);
            p.ws_lens = bump(off, (uint64_t)sigma * 4);
            p.ws_ktab = bump(off, (uint64_t)sigma * 4);
            p.ws_scounts = bump(off, (uint64_t)sigma * 8);
        }
        p.ws_bytes = off;
        return WT_OK;
    }
    if (kind == WT_KIND_WM && !p.levelwise) {
        p.tau = p.wm.tau;
        p.ws_wm = bump(off, p.wm.ws_bytes);
    } else {
        p.tau = 1;
        p.ws_keys_a = bump(off, std::max<uint64_t>(n, 1) * 4);
        p.ws_keys_b = bump(off, std::max<uint64_t>(n, 1) * 4);
    }
    if (is_tree(kind)) {
        p.ws_nodes_a = bump(off, std::max<uint64_t>(n, 1) * 4);
        p.ws_nodes_b = bump(off, std::max<uint64_t>(n, 1) * 4);
        p.ws_counts = bump(off, (uint64_t)sigma * 8);
        p.ws_nt_start = bump(off, p.node_bound * 4);
        p.ws_nt_cstart = bump(off, p.node_bound * d * 4);
        p.ws_nt_child = bump(off, p.node_bound * d * 4);
    }
    if (kind == WT_KIND_SHAPED) {
        p.ws_codes = bump(off, (uint64_t)sigma * 4);
        p.ws_lens = bump(off, (uint64_t)sigma * 4);
    }
    p.ws_bytes = off;
    return WT_OK;
}

const char* kind_name(int kind)
{
    switch (kind) {
    case WT_KIND_WT: return "tree";
    case WT_KIND_WM: return "matrix";
    case WT_KIND_SHAPED: return "shaped";
    case WT_KIND_MULTIARY: return "multiary";
    default: return "?";
    }
}

// the plan, and with WT_TRACE set its figures on stderr: the path, the
// passes (tau, chunks K of C keys in tiles of 8192), the workspace and every
// level's array offsets in the image
int make_plan(int kind, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
              const wt_tuning* tune, Plan& p)
{
    const int rc = make_plan_impl(kind, n, sigma, sym_bytes, shape, tune, p);
    if (!wv_trace_on()) return rc;
    if (rc) {
        wv_trace("plan %s n=%llu sigma=%u sym_bytes=%u: %s", kind_name(kind), (unsigned long long)n, sigma,
                 sym_bytes, wt_strerror(rc));
        return rc;
    }
    const wv_wm_plan& m = p.wm.enabled ? p.wm : p.wmb;
    const char* path = p.direct_tree ? "one-pass tree order"
                       : (kind != WT_KIND_WM && p.dev_runs) ? "matrix passes + device runs + permutation"
                       : m.enabled ? "matrix passes" : "level by level";
    wv_trace("plan %s n=%llu sigma=%u sym_bytes=%u levels=%u key_bits=%u path=%s", kind_name(kind),
             (unsigned long long)n, sigma, sym_bytes, p.nlevels, p.key_bits, path);
    if (m.enabled)
        wv_trace("  passes: tau=%u passes=%u chunks K=%u of C=%u keys (%u tiles) workspace=%llu", m.tau,
                 (m.L + m.tau - 1) / m.tau, m.K, m.C, m.C / 8192u, (unsigned long long)p.ws_bytes);
    if (p.h1)
        wv_trace("  split at %u key bits: matrix A over every symbol's top bits, matrix B over the %llu "
                 "symbols with longer codes (tau=%u)", p.h1, (unsigned long long)p.nlong, p.wmb.tau);
    else
        wv_trace("  workspace=%llu", (unsigned long long)p.ws_bytes);
    for (uint32_t l = 0; l < p.nlevels; l++) {
        const wv_level& L = p.lay.lv[l];
        wv_trace("  level %u: n=%llu bits@%llu rank@%llu sel0@%llu sel1@%llu nsel=%llu", l,
                 (unsigned long long)L.n, (unsigned long long)L.bits_off, (unsigned long long)L.rank_off,
                 (unsigned long long)L.sel0_off, (unsigned long long)L.sel1_off, (unsigned long long)L.nsel);
    }
    wv_trace("  image=%llu bytes", (unsigned long long)p.lay.image_bytes);
    return rc;
}


// ---- host node tables ----------------------------------------------------------

struct HostNodes {
    std::vector<uint32_t> start, child_start, child;
};

// Balanced trees (binary D = 1, or multiary): node = nonempty prefix of the
// top D*beta key bits; every level keeps all n symbols, so a node's start is
// the number of symbols with a smaller prefix.
int balanced_nodes(const std::vector<uint64_t>& counts, uint32_t sigma, uint32_t Lb, uint32_t D, uint32_t M,
                   HostNodes& H)
{
    const uint32_t d = 1u << D;
    std::vector<std::vector<uint64_t>> pc(M), st(M);
    std::vector<std::vector<uint32_t>> id(M);
    uint32_t next = 0;
    for (uint32_t be = 0; be < M; be++) {
        const uint32_t sh = Lb - D * be;
        const uint64_t size = sh >= 64 ? 1 : (((uint64_t)(sigma - 1) >> sh) + 1);
        pc[be].assign(size, 0);
        for (uint32_t x = 0; x < sigma; x++) pc[be][sh >= 64 ? 0 : ((uint64_t)x >> sh)] += counts[x];
        st[be].assign(size, 0);
        id[be].assign(size, WV_NONE);
        uint64_t run = 0;
        for (uint64_t q = 0; q < size; q++) {
            st[be][q] = run;
            run += pc[be][q];
            if (pc[be][q] || (be == 0)) id[be][q] = next++;
        }
    }
    H.start.assign(next, 0);
    H.child_start.assign((uint64_t)next * d, 0);
    H.child.assign((uint64_t)next * d, WV_NONE);
    for (uint32_t be = 0; be < M; be++) {
        for (uint64_t q = 0; q < pc[be].size(); q++) {
            const uint32_t k = id[be][q];
            if (k == WV_NONE) continue;
            H.start[k] = (uint32_t)st[be][q];
            for (uint32_t g = 0; g < d; g++) {
                uint32_t c = WV_LEAF;
                uint64_t cs = 0;
                if (be + 1 < M) {
                    const uint64_t q2 = q * d + g;
                    c = WV_NONE;
                    if (q2 < pc[be + 1].size() && pc[be + 1][q2]) {
                        c = id[be + 1][q2];
                        cs = st[be + 1][q2];
                    }
                }
                H.child[(uint64_t)k * d + g] = c;
                H.child_start[(uint64_t)k * d + g] = (uint32_t)cs;
            }
        }
    }
    return WT_OK;
}

// Shaped tree (Sec. 4.3): internal nodes are the proper codeword prefixes,
// ordered by (level, prefix); the start of a node on its level is the number
// of symbols of that level under smaller prefixes.  Also fills the image's
// node-table records.  Built level by level from the codewords in padded
// order, in which the prefixes of one length come out sorted.
int shaped_nodes(const wt_shape& sh, uint32_t sigma, HostNodes& H, std::vector<uint8_t>& rec)
{
    const uint32_t D = std::max(sh.arity_log2, 1u), d = 1u << D;
    const uint64_t RB = wv_node_bytes(D >= 2 ? D : 1);
    uint32_t h = 0;
    for (uint32_t x = 0; x < sigma; x++) h = std::max(h, sh.code_len[x]);
    std::vector<Coded> cs;
    uint64_t N = 0;
    int rc = sorted_codes(sh, sigma, h, cs, &N, D);
    if (rc) return rc;
    // symbols before every position of the key order
    std::vector<uint64_t> pc(cs.size() + 1, 0);
    for (size_t i = 0; i < cs.size(); i++) pc[i + 1] = pc[i] + sh.counts[cs[i].sym];
    H.start.assign(N, 0);
    H.child_start.assign(d * N, 0);
    H.child.assign(d * N, WV_NONE);
    rec.assign(N * RB, 0);
    // level by level, nodes in key order: a node is the range of codewords
    // sharing its prefix; its children split the range by the next digit
    // (the keys of one node are sorted by it), a child holding one codeword
    // that ends there is that symbol's leaf
    struct Node { uint32_t a, b; uint64_t start; };
    std::vector<Node> cur, nxt;
    if (!cs.empty()) cur.push_back(Node{0, (uint32_t)cs.size(), 0});
    uint64_t base = 0;
    std::vector<uint32_t> lo(d), hi(d), ch(d);
    for (uint32_t l = 0; l < h && !cur.empty(); l++) {
        const uint64_t nbase = base + cur.size();
        if (nbase > N) return WT_EINVAL;
        const uint32_t shift = D * (h - 1 - l);   // digit l of a padded key
        nxt.clear();
        uint64_t nrun = 0;
        for (uint64_t k = 0; k < cur.size(); k++) {
            const Node nd = cur[k];
            const uint64_t t = base + k;
            const uint64_t cnt = pc[nd.b] - pc[nd.a];
            uint32_t a = nd.a;
            for (uint32_t g = 0; g < d; g++) {
                const uint32_t m = g + 1 < d
                    ? (uint32_t)(std::partition_point(cs.begin() + a, cs.begin() + nd.b,
                                                      [&](const Coded& c) { return ((c.key >> shift) & (d - 1)) <= g; }) -
                                 cs.begin())
                    : nd.b;
                lo[g] = a;
                hi[g] = m;
                a = m;
            }
            for (uint32_t g = 0; g < d; g++) {
                uint32_t c = WV_NONE;
                uint64_t cst = 0;
                if (hi[g] - lo[g] == 1 && cs[lo[g]].len == l + 1) {
                    c = WV_LEAF | cs[lo[g]].sym;
                } else if (hi[g] > lo[g]) {
                    const uint64_t id = nbase + nxt.size();
                    if (id >= N) return WT_EINVAL;
                    c = (uint32_t)id;
                    cst = nrun;
                    nxt.push_back(Node{lo[g], hi[g], nrun});
                    nrun += pc[hi[g]] - pc[lo[g]];
                }
                ch[g] = c;
                H.child[(uint64_t)d * t + g] = c;
                H.child_start[(uint64_t)d * t + g] = (uint32_t)cst;
            }
            H.start[t] = (uint32_t)nd.start;
            uint8_t* e = rec.data() + t * RB;
            const uint32_t lev = l, pr = l ? (uint32_t)(cs[nd.a].key >> (D * (h - l))) : 0u;
            std::memcpy(e + 0, &nd.start, 8);
            std::memcpy(e + 8, &cnt, 8);
            if (D == 1) {
                std::memcpy(e + 16, &ch[0], 4);
                std::memcpy(e + 20, &ch[1], 4);
                std::memcpy(e + 24, &lev, 4);
                std::memcpy(e + 28, &pr, 4);
            } else {
                std::memcpy(e + 16, &lev, 4);
                std::memcpy(e + 20, &pr, 4);
                std::memcpy(e + 24, ch.data(), 4ull * d);
            }
        }
        base = nbase;
        cur.swap(nxt);
    }
    if (base != N || !cur.empty()) return WT_EINVAL;
    return WT_OK;
}

template <typename T>
T* at(void* base, uint64_t off) { return (T*)((uint8_t*)base + off); }

wv_lw_args lw_args(const Plan& p, const void* S, void* out, void* ws)
{
    wv_lw_args a{};
    a.kind = p.kind;
    a.arity_log2 = p.D;
    a.key_bits = p.key_bits;
    a.nlevels = p.nlevels;
    a.S = S;
    a.image = (uint8_t*)out;
    a.lay = &p.lay;
    a.keys_a = at<uint32_t>(ws, p.ws_keys_a);
    a.keys_b = at<uint32_t>(ws, p.ws_keys_b);
    a.nodes_a = at<uint32_t>(ws, p.ws_nodes_a);
    a.nodes_b = at<uint32_t>(ws, p.ws_nodes_b);
    a.dir.sb_ones = at<uint32_t>(ws, p.ws_sb_ones);
    a.dir.sb_pre = at<uint64_t>(ws, p.ws_sb_pre);
    a.dir.partial = at<uint64_t>(ws, p.ws_partial);
    a.dir.total = at<uint64_t>(ws, p.ws_scalars + 8);
    a.mdir.rng_cnt = a.dir.sb_ones;
    a.mdir.rng_pre = a.dir.sb_pre;
    a.mdir.partial = a.dir.partial;
    a.mdir.totals = at<uint64_t>(ws, p.ws_mtot);
    a.zl = at<uint64_t>(ws, p.ws_scalars);
    a.nt.start = at<uint32_t>(ws, p.ws_nt_start);
    a.nt.child_start = at<uint32_t>(ws, p.ws_nt_cstart);
    a.nt.child = at<uint32_t>(ws, p.ws_nt_child);
    a.codes = at<uint32_t>(ws, p.ws_codes);
    a.lens = at<uint32_t>(ws, p.ws_lens);
    return a;
}

int check_buffers(const Plan& p, const void* S, void* out, size_t out_bytes, void* ws, size_t ws_bytes)
{
    if ((!S && p.n) || !out || (!ws && p.ws_bytes)) return WT_EINVAL;
    // the kernels read S and the workspace in 16-byte pieces
    if (((uintptr_t)S | (uintptr_t)out | (uintptr_t)ws) & 15u) return WT_EINVAL;
    if (out_bytes < p.lay.image_bytes || ws_bytes < p.ws_bytes) return WT_ENOSPC;
    return WT_OK;
}

// Balanced or shaped binary tree gathered from matrix levels: validate S and
// count its symbols, derive every level's runs on the host, build the matrix
// levels of the (padded) keys, move the runs, then the directories.
// Events for stream forks and joins, kept in a pool for the process
std::mutex& event_mu()
{
    static std::mutex m;
    return m;
}
std::vector<hipEvent_t>& event_pool()
{
    static std::vector<hipEvent_t> v;
    return v;
}
hipEvent_t take_event()
{
    {
        std::lock_guard<std::mutex> lk(event_mu());
        auto& v = event_pool();
        if (!v.empty()) {
            hipEvent_t e = v.back();
            v.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
}
void give_event(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(event_mu());
    event_pool().push_back(e);
}

// Balanced binary and multiary trees: the matrix passes over the symbols (and
// the digit strings of a multiary tree), every level's runs derived on the
// device from the symbol counts, the gather to tree order, the directories.
// Every step is a launch on `s`: nothing is copied to or from the host and
// nothing waits, so the build can be captured in a graph.
int build_balanced_dev(const Plan& p, const void* S, uint8_t* img, uint8_t* ws, bool prof, hipStream_t s)
{
    const uint64_t n = p.n;
    const uint32_t sigma = p.sigma, K = p.key_bits;
    const bool multi = p.kind == WT_KIND_MULTIARY;
    const uint32_t D = multi ? p.D : 1u, T = multi ? p.nlevels : K;
    uint64_t* dcounts = at<uint64_t>(ws, p.ws_counts);
    WV_TIMED(prof, s, "validate", WV_CHECK(wv_validate(S, n, p.sym_bytes, sigma, img, dcounts, s)));
    if (multi) {
        uint8_t* timg = at<uint8_t>(ws, p.ws_tmpimg);
        const uint64_t *zpre = nullptr, *ztot = nullptr;
        if (D == 4) {
            wv_dir_scratch unused{};
            WV_CHECK(wv_wm_run(p.wm, S, timg, p.tlay, at<uint8_t>(ws, p.ws_wm), unused, s));
        } else {
            uint64_t* lw[WV_MAX_LEVELS];
            for (uint32_t l = 0; l < K; l++) lw[l] = (uint64_t*)(timg + p.tlay.lv[l].bits_off);
            WV_CHECK(wv_wm_levels(p.wm, S, lw, nullptr, at<uint8_t>(ws, p.ws_wm), s));
            if (D == 2) {
                wv_digit_words dw{};
                for (uint32_t t = 0; t < T; t++) dw.w[t] = lw[2 * t];
                uint32_t* cnt = at<uint32_t>(ws, p.ws_sb_ones);
                uint64_t* pre = at<uint64_t>(ws, p.ws_sb_pre);
                uint64_t* tot = at<uint64_t>(ws, p.ws_mtot);
                WV_TIMED(prof, s, "tree_digits", WV_CHECK(wv_digit_zero_counts(dw, n, T, cnt, s)));
                WV_TIMED(prof, s, "tree_digits",
                         WV_CHECK(wv_scan_u32(cnt, pre, wv_digit_blocks(n), T, at<uint64_t>(ws, p.ws_partial), tot, s)));
                zpre = pre;
                ztot = tot;
            }
        }
        wv_digit_set ds{};
        for (uint32_t t = 0; t < T; t++) {
            for (uint32_t k = 0; k < D; k++) {
                ds.lv[t].words[k] = (const uint64_t*)(timg + p.tlay.lv[t * D + k].bits_off);
                ds.lv[t].dir[k] = (const uint64_t*)(timg + p.tlay.lv[t * D + k].rank_off);
            }
            ds.out[t] = at<uint64_t>(ws, p.ws_digits + t * p.dstride);
        }
        WV_TIMED(prof, s, "tree_digits", WV_CHECK(wv_tree_digits(ds, T, n, D, zpre, ztot, s)));
    } else {
        uint64_t* lw[WV_MAX_LEVELS];
        for (uint32_t l = 0; l < K; l++) lw[l] = at<uint64_t>(ws, p.ws_tmp + l * p.tmp_stride);
        WV_CHECK(wv_wm_levels(p.wm, S, lw, nullptr, at<uint8_t>(ws, p.ws_wm), s));
    }
    uint8_t* gws = at<uint8_t>(ws, p.ws_group);
    WV_TIMED(prof, s, "tree_runs", WV_CHECK(wv_tree_group_runs(dcounts, sigma, K, gws, p.gz, s)));
    wv_group_level lv[WV_MAX_LEVELS];
    for (uint32_t t = 0; t < T; t++) {
        lv[t].dst = (uint64_t*)(img + p.lay.lv[t].bits_off);
        lv[t].src = multi ? at<uint64_t>(ws, p.ws_digits + t * p.dstride) : at<uint64_t>(ws, p.ws_tmp + t * p.tmp_stride);
        lv[t].nbits = p.lay.lv[t].n * D;
        lv[t].l = t * D;
        // multiary: the sub-range counters follow the range counters
        lv[t].sub = multi ? (uint16_t*)(img + p.lay.lv[t].rank_off + (wv_mranges(p.lay.lv[t].n, D) + 1) * (8ull << D))
                          : nullptr;
    }
    const wv_mdir_scratch md{at<uint32_t>(ws, p.ws_sb_ones), at<uint64_t>(ws, p.ws_sb_pre),
                             at<uint64_t>(ws, p.ws_partial), at<uint64_t>(ws, p.ws_mtot)};
    const wv_perm_counts pc{md.rng_cnt, n, D, T};
    WV_TIMED(prof, s, "tree_perm", WV_CHECK(wv_tree_permute_groups(lv, T, K, D, gws, p.gz, multi ? &pc : nullptr, s)));
    if (multi) WV_TIMED(prof, s, "mcounters", WV_CHECK(wv_multiary_ranges(img, p.lay.lv, T, D, md, s)));
    else WV_CHECK(wv_span_directory(img, p.lay, 0, K, at<uint8_t>(ws, p.ws_wm + p.wm.off_dir), p.wm.dir, s, prof));
    return WT_OK;
}

int build_from_matrix(const Plan& p, const void* S, const wt_shape* shape, uint8_t* img, uint8_t* ws, bool prof,
                      hipStream_t s)
{
    if (p.dev_runs) return build_balanced_dev(p, S, img, ws, prof, s);
    const uint64_t n = p.n;
    const uint32_t sigma = p.sigma, K = p.key_bits;
    const bool shaped = p.kind == WT_KIND_SHAPED, multi = p.kind == WT_KIND_MULTIARY;
    // levels of D-bit digits: multiary trees, and shaped trees over digits
    // (levels of different lengths; their counters are taken during the
    // gather all the same)
    const bool digits = multi || (shaped && p.D >= 2);
    const uint32_t D = digits ? p.D : 1u, T = digits ? p.nlevels : K;
    // 1. symbol counts (and status).  A shaped tree takes its counts from the
    // shape, which fixes the level sizes, and the device only checks them
    // (image status); a balanced tree over more than WV_GROUP_MAX_BITS key
    // bits reads them back to lay out its runs on the host (waited for in
    // step 3)
    const bool readback = !shaped;
    uint64_t* dcounts = at<uint64_t>(ws, p.ws_counts);
    WV_TIMED(prof, s, "validate", WV_CHECK(wv_validate(S, n, p.sym_bytes, sigma, img, dcounts, s)));
    // [status word][counts], pinned when possible (else a pageable array)
    PinnedBuf pin(readback ? ((uint64_t)sigma + 1) * 8 : 0, s);
    std::vector<uint64_t> unpinned(readback && !pin.get() ? (uint64_t)sigma + 1 : 0);
    uint64_t* hc = pin.get() ? (uint64_t*)pin.get() : unpinned.data();
    hipEvent_t have_counts = nullptr;
    struct EventGuard {
        hipEvent_t e;
        ~EventGuard()
        {
            if (e) (void)hipEventDestroy(e);
        }
    } guard{nullptr};
    if (readback) {
        hc[0] = 0;
        WV_CHECK(hipMemcpyAsync(hc + 1, dcounts, (uint64_t)sigma * 8, hipMemcpyDeviceToHost, s));
        WV_CHECK(hipMemcpyAsync(hc, img + 36, 4, hipMemcpyDeviceToHost, s));
        WV_CHECK(hipEventCreateWithFlags(&have_counts, hipEventDisableTiming));
        guard.e = have_counts;
        WV_CHECK(hipEventRecord(have_counts, s));
    }
    // fork / join of the side stream (split shaped trees): events from a pool,
    // given back when the call returns (a wait already queued on an event is
    // not affected when the event is recorded again, and destroying an event
    // that the device has not reached yet would hold the host)
    struct ForkEvents {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~ForkEvents()
        {
            for (hipEvent_t x : e)
                if (x) give_event(x);
        }
    } fork;
    if (p.h1 && p.nlong)
        for (hipEvent_t& x : fork.e)
            if (!(x = take_event())) return WT_EHIP;

    // 2. the matrix levels need no counts: launch them now, so that they run
    // while the host lays out the tree
    std::vector<uint32_t> c32, l32, ktab;
    // host buffers of the uploads: pinned (pooled) when possible, released
    // to the pool once the stream has passed the copies
    PinnedBuf up_codes(shaped ? (p.ws_scounts - p.ws_codes + (uint64_t)sigma * 8) : 0, s);
    std::vector<uint8_t> up_codes_v, up_late_v;
    const void* keys = S;
    if (shaped) {
        // codeword lengths in bits (digits of D bits)
        c32.resize(sigma);
        l32.resize(sigma);
        for (uint32_t x = 0; x < sigma; x++) {
            l32[x] = shape->code_len[x] * p.D;
            c32[x] = l32[x] ? (uint32_t)shape->codes[x] : 0u;
        }
        if (p.h1) wv_split_table(c32.data(), l32.data(), sigma, K, p.h1, ktab);   // top h1 bits of every codeword
        else wv_key_table(c32.data(), l32.data(), sigma, K, ktab);                // every codeword padded to K bits
        // codes, lengths (and key table) and the shape's counts in the
        // workspace layout, one copy; the device checks its counts against
        // the shape's (image status)
        const uint64_t span = p.ws_scounts - p.ws_codes + (uint64_t)sigma * 8;
        if (!up_codes.get()) up_codes_v.resize(span);
        uint8_t* hb = up_codes.get() ? (uint8_t*)up_codes.get() : up_codes_v.data();
        std::memcpy(hb, c32.data(), (uint64_t)sigma * 4);
        std::memcpy(hb + (p.ws_lens - p.ws_codes), l32.data(), (uint64_t)sigma * 4);
        std::memcpy(hb + (p.ws_ktab - p.ws_codes), ktab.data(), (uint64_t)sigma * 4);
        std::memcpy(hb + (p.ws_scounts - p.ws_codes), shape->counts, (uint64_t)sigma * 8);
        if (up_codes.get()) WV_CHECK(wv_upload(at<void>(ws, p.ws_codes), hb, span, s));
        else WV_CHECK(hipMemcpyAsync(at<void>(ws, p.ws_codes), hb, span, hipMemcpyHostToDevice, s));
        WV_CHECK(wv_check_counts(dcounts, at<uint64_t>(ws, p.ws_scounts), sigma, img, s));
        const uint32_t* dc = at<uint32_t>(ws, p.ws_codes);
        const uint32_t* dl = at<uint32_t>(ws, p.ws_lens);
        if (p.h1) {
            // the 16-bit keys, then the long codewords compacted
            const uint32_t* dk = at<uint32_t>(ws, p.ws_ktab);
            uint64_t* boff = at<uint64_t>(ws, p.ws_boff);
            WV_TIMED(prof, s, "tree_keys",
                     WV_CHECK(wv_tree_keys_split(S, n, p.sym_bytes, sigma, dk, at<uint16_t>(ws, p.ws_tkeys),
                                                 at<uint32_t>(ws, p.ws_bcnt), at<uint16_t>(ws, p.ws_lmask), s)));
            WV_TIMED(prof, s, "tree_keys",
                     WV_CHECK(wv_scan_u32(at<uint32_t>(ws, p.ws_bcnt), boff, p.nkblocks, 1, at<uint64_t>(ws, p.ws_bpart),
                                          boff + p.nkblocks, s)));
            WV_TIMED(prof, s, "tree_keys",
                     WV_CHECK(wv_tree_long_keys(S, n, p.sym_bytes, dc, dl, K, boff, at<uint16_t>(ws, p.ws_lmask),
                                                at<uint32_t>(ws, p.ws_lkeys), p.nlong, s)));
        } else {
            WV_TIMED(prof, s, "tree_keys",
                     WV_CHECK(wv_tree_keys(S, n, p.sym_bytes, sigma, at<uint32_t>(ws, p.ws_ktab),
                                           at<uint32_t>(ws, p.ws_tkeys), s)));
        }
        keys = at<void>(ws, p.ws_tkeys);
    }
    if (digits) {
        // the matrix levels in the workspace, then the digits: 2-bit digits
        // need only the zeros before every 256-word block of the levels 2t,
        // 16-ary digits query the matrix's rank directories.  A split shaped
        // tree takes digit levels t < TA from matrix A (n symbols) and the
        // others from matrix B (the long-code symbols), built on the side
        // stream meanwhile.
        const uint32_t TA = p.h1 ? p.h1 / D : T;
        auto run_matrix = [&](const wv_wm_plan& wp, const void* in, uint8_t* mimg, const wv_layout_out& lay,
                              uint32_t levels, uint8_t* mws, hipStream_t st) -> hipError_t {
            if (D == 4) {
                wv_dir_scratch unused{};
                return wv_wm_run(wp, in, mimg, lay, mws, unused, st);
            }
            uint64_t* lw[WV_MAX_LEVELS];
            for (uint32_t l = 0; l < levels; l++) lw[l] = (uint64_t*)(mimg + lay.lv[l].bits_off);
            return wv_wm_levels(wp, in, lw, nullptr, mws, st);
        };
        auto digit_strings = [&](const uint8_t* mimg, const wv_layout_out& lay, uint64_t m, uint32_t t0,
                                 uint32_t nt) -> hipError_t {
            const uint64_t *zpre = nullptr, *ztot = nullptr;
            if (D == 2) {
                // scratch of the digit counters, not used before the gather
                wv_digit_words dw{};
                for (uint32_t t = 0; t < nt; t++) dw.w[t] = (const uint64_t*)(mimg + lay.lv[2 * (t0 + t)].bits_off);
                uint32_t* cnt = at<uint32_t>(ws, p.ws_sb_ones);
                uint64_t* pre = at<uint64_t>(ws, p.ws_sb_pre);
                uint64_t* tot = at<uint64_t>(ws, p.ws_mtot);
                hipError_t e = wv_digit_zero_counts(dw, m, nt, cnt, s);
                if (e == hipSuccess) e = wv_scan_u32(cnt, pre, wv_digit_blocks(m), nt, at<uint64_t>(ws, p.ws_partial), tot, s);
                if (e != hipSuccess) return e;
                zpre = pre;
                ztot = tot;
            }
            wv_digit_set ds{};
            for (uint32_t t = 0; t < nt; t++) {
                for (uint32_t k = 0; k < D; k++) {
                    ds.lv[t].words[k] = (const uint64_t*)(mimg + lay.lv[(t0 + t) * D + k].bits_off);
                    ds.lv[t].dir[k] = (const uint64_t*)(mimg + lay.lv[(t0 + t) * D + k].rank_off);
                }
                ds.out[t] = at<uint64_t>(ws, p.ws_digits + (t0 + t) * p.dstride);
            }
            return wv_tree_digits(ds, nt, m, D, zpre, ztot, s);
        };
        uint8_t* timg = at<uint8_t>(ws, p.ws_tmpimg);
        const bool two = p.h1 && p.nlong;
        // matrix B on the side stream (on `s` when there is none), forked
        // after the keys, joined before its digits are read
        hipStream_t s2 = two ? wv_side_stream() : nullptr;
        if (two) {
            hipStream_t sb = s2 ? s2 : s;
            wv_wm_plan pb = p.wmb;
            pb.profile = false;
            if (s2) {
                WV_CHECK(hipEventRecord(fork.e[0], s));
                WV_CHECK(hipStreamWaitEvent(s2, fork.e[0], 0));
            }
            WV_TIMED(prof, sb, "side_matrix",
                     WV_CHECK(run_matrix(pb, at<void>(ws, p.ws_lkeys), at<uint8_t>(ws, p.ws_timgb), p.tlayb, K,
                                         at<uint8_t>(ws, p.ws_wmb), sb)));
            if (s2) WV_CHECK(hipEventRecord(fork.e[1], s2));
        }
        WV_CHECK(run_matrix(p.wm, keys, timg, p.tlay, p.h1 ? p.h1 : K, at<uint8_t>(ws, p.ws_wm), s));
        WV_TIMED(prof, s, "tree_digits", WV_CHECK(digit_strings(timg, p.tlay, n, 0, TA)));
        if (two) {
            if (s2) WV_CHECK(hipStreamWaitEvent(s, fork.e[1], 0));
            WV_TIMED(prof, s, "tree_digits",
                     WV_CHECK(digit_strings(at<uint8_t>(ws, p.ws_timgb), p.tlayb, p.nlong, TA, T - TA)));
        }
    } else if (p.h1) {
        // S itself was validated above; the keys need no check
        // the big matrix first, then the small matrix of the long codes on a
        // side stream: its short, launch-bound passes are queued while the
        // big matrix's first pass runs and fill in beside it (forked after the
        // keys, joined before anything reads its levels)
        hipStream_t s2 = p.nlong ? wv_side_stream() : nullptr;
        if (s2) WV_CHECK(hipEventRecord(fork.e[0], s));
        uint64_t* lwa[WV_MAX_LEVELS];
        for (uint32_t l = 0; l < p.h1; l++) lwa[l] = at<uint64_t>(ws, p.ws_tmp + l * p.tmp_stride);
        WV_CHECK(wv_wm_levels(p.wm, keys, lwa, nullptr, at<uint8_t>(ws, p.ws_wm), s));
        if (p.nlong) {
            uint64_t* lwb[WV_MAX_LEVELS];
            for (uint32_t l = 0; l < K; l++) lwb[l] = at<uint64_t>(ws, p.ws_btmp + l * p.btmp_stride);
            const void* lk = at<void>(ws, p.ws_lkeys);
            if (s2) {
                // timed as a whole: per-kernel events on the side stream
                // would count the time its kernels wait for the CUs
                wv_wm_plan pb = p.wmb;
                pb.profile = false;
                WV_CHECK(hipStreamWaitEvent(s2, fork.e[0], 0));
                WV_TIMED(prof, s2, "side_matrix", WV_CHECK(wv_wm_levels(pb, lk, lwb, nullptr, at<uint8_t>(ws, p.ws_wmb), s2)));
                WV_CHECK(hipEventRecord(fork.e[1], s2));
            } else {
                WV_CHECK(wv_wm_levels(p.wmb, lk, lwb, nullptr, at<uint8_t>(ws, p.ws_wmb), s));
            }
        }
        if (s2) WV_CHECK(hipStreamWaitEvent(s, fork.e[1], 0));
    } else {
        uint64_t* lw[WV_MAX_LEVELS];
        for (uint32_t l = 0; l < K; l++) lw[l] = at<uint64_t>(ws, p.ws_tmp + l * p.tmp_stride);
        WV_CHECK(wv_wm_levels(p.wm, keys, lw, (uint32_t*)(img + 36), at<uint8_t>(ws, p.ws_wm), s));
    }

    // 3. the counts (a shaped tree's from the shape, nothing to wait for)
    uint32_t status = 0;
    std::vector<uint64_t> counts;
    if (readback) {
        WV_CHECK(hipEventSynchronize(have_counts));
        status = (uint32_t)hc[0];
        counts.assign(hc + 1, hc + 1 + sigma);
        pin.idle();
    } else {
        counts.assign(shape->counts, shape->counts + sigma);
    }
    int rc = status ? WT_ERANGE : WT_OK;
    // work already launched writes into the caller's buffers: on an error a
    // shaped build leaves it queued (its uploads retire with the stream), the
    // other path lets it finish
    auto fail = [&](int code) {
        if (shaped && !up_codes_v.size() && !up_late_v.size()) {
            up_codes.retire(s);
            return code;
        }
        (void)hipStreamSynchronize(s);
        up_codes.idle();
        return code;
    };
    std::vector<uint8_t> rec, code_rec;
    if (!rc && shaped) {
        HostNodes H;
        rc = shaped_nodes(*shape, sigma, H, rec);
        code_rec.assign((uint64_t)sigma * WV_CODE_BYTES, 0);
        for (uint32_t x = 0; x < sigma; x++) {
            const uint64_t c = c32[x];
            const uint32_t len = shape->code_len[x];   // in digits
            std::memcpy(code_rec.data() + (uint64_t)x * WV_CODE_BYTES, &c, 8);
            std::memcpy(code_rec.data() + (uint64_t)x * WV_CODE_BYTES + 8, &len, 4);
        }
    }
    // 4. every level's runs, from the counts
    std::vector<wv_perm_seg> segs;
    std::vector<uint64_t> seg0;
    if (!rc) {
        wv_tree_segments(counts, K, shaped ? c32.data() : nullptr, shaped ? l32.data() : nullptr, segs, seg0);
        if (p.h1) {
            // levels from h1 on hold the long-code symbols only, as matrix B
            std::vector<uint64_t> cl(counts);
            for (uint32_t x = 0; x < sigma; x++)
                if (l32[x] <= p.h1) cl[x] = 0;
            std::vector<wv_perm_seg> sb;
            std::vector<uint64_t> s0b;
            wv_tree_segments(cl, K, c32.data(), l32.data(), sb, s0b);
            segs.resize(seg0[p.h1]);
            for (uint32_t l = p.h1; l < K; l++) {
                seg0[l] = segs.size();
                segs.insert(segs.end(), sb.begin() + s0b[l], sb.begin() + s0b[l + 1]);
            }
            seg0[K] = segs.size();
        }
        // tree level t: matrix level t (binary), or digit level t from matrix
        // level t*D with every run D bits per symbol (digit levels)
        if (digits) {
            std::vector<wv_perm_seg> ms;
            std::vector<uint64_t> m0(T + 1, 0);
            for (uint32_t t = 0; t < T; t++) {
                m0[t] = ms.size();
                for (uint64_t k = seg0[t * D]; k < seg0[t * D + 1]; k++)
                    ms.push_back(wv_perm_seg{segs[k].dst * D, segs[k].src * D, segs[k].len * D});
            }
            m0[T] = ms.size();
            segs.swap(ms);
            seg0.swap(m0);
        }
        if (segs.size() > p.seg_bound) rc = WT_EUNSUP;
    }
    if (rc) return fail(rc);
    std::vector<wv_perm_level> lv(T);
    for (uint32_t l = 0; l < T; l++) {
        lv[l].dst = (uint64_t*)(img + p.lay.lv[l].bits_off);
        lv[l].src = digits ? at<uint64_t>(ws, p.ws_digits + l * p.dstride)
                  : (p.h1 && l >= p.h1) ? at<uint64_t>(ws, p.ws_btmp + l * p.btmp_stride)
                                        : at<uint64_t>(ws, p.ws_tmp + l * p.tmp_stride);
        lv[l].nbits = p.lay.lv[l].n * D;
        lv[l].seg0 = seg0[l];
        lv[l].nseg = seg0[l + 1] - seg0[l];
        lv[l].sub = nullptr;
        // digit levels: the sub-range counters follow the range counters
        if (digits) lv[l].sub = (uint16_t*)(img + p.lay.lv[l].rank_off + (wv_mranges(p.lay.lv[l].n, D) + 1) * (8ull << D));
    }
    std::vector<uint32_t> tile0, tile_seg;
    wv_tree_tiles(lv, segs, digits, tile0, tile_seg);
    if (tile_seg.size() > p.tile_bound) return fail(WT_EUNSUP);
    // descriptors, runs and tiles in one copy; the node and code tables of a
    // shaped tree behind them in the same host buffer
    const uint64_t seg_at = wv_round256(WV_MAX_LEVELS * sizeof(wv_perm_level));
    const uint64_t tile_at = seg_at + wv_round256(segs.size() * sizeof(wv_perm_seg));
    const uint64_t stage_bytes = tile_at + tile_seg.size() * 4;
    const uint64_t rec_at = wv_round256(stage_bytes), code_at = rec_at + wv_round256(rec.size());
    const uint64_t late_bytes = code_at + code_rec.size();
    PinnedBuf late(late_bytes, s);
    if (!late.get()) up_late_v.resize(late_bytes);
    uint8_t* stage = late.get() ? (uint8_t*)late.get() : up_late_v.data();
    std::memcpy(stage, lv.data(), T * sizeof(wv_perm_level));
    if (!segs.empty()) std::memcpy(stage + seg_at, segs.data(), segs.size() * sizeof(wv_perm_seg));
    if (!tile_seg.empty()) std::memcpy(stage + tile_at, tile_seg.data(), tile_seg.size() * 4);
    if (!rec.empty()) std::memcpy(stage + rec_at, rec.data(), rec.size());
    if (!code_rec.empty()) std::memcpy(stage + code_at, code_rec.data(), code_rec.size());
    uint8_t* dsegs = at<uint8_t>(ws, p.ws_segs);
    auto upload = [&](void* dst, const void* src, uint64_t bytes) {
        return late.get() ? wv_upload(dst, src, bytes, s) : hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    WV_CHECK(upload(dsegs, stage, stage_bytes));
    const wv_perm_level* dlv = (const wv_perm_level*)dsegs;
    const wv_perm_seg* dseg = (const wv_perm_seg*)(dsegs + seg_at);
    const uint32_t* dtile = (const uint32_t*)(dsegs + tile_at);
    if (shaped) {
        if (!rec.empty())
            WV_CHECK(upload(img + p.lay.nodes_off, stage + rec_at, rec.size()));
        WV_CHECK(upload(img + p.lay.codes_off, stage + code_at, code_rec.size()));
    }

    // 5. runs to tree order, then the directories
    // digit levels: the gather also counts digits per range and sub-range
    // (levels shorter than the first leave rows of the range counts that
    // the scan must read as zero)
    const wv_mdir_scratch md{at<uint32_t>(ws, p.ws_sb_ones), at<uint64_t>(ws, p.ws_sb_pre),
                             at<uint64_t>(ws, p.ws_partial), at<uint64_t>(ws, p.ws_mtot)};
    const wv_perm_counts pc{md.rng_cnt, n, D, T};
    if (digits && !multi) {
        const uint64_t cells = wv_mranges(n, D) * T * (1ull << D);
        WV_TIMED(prof, s, "mcounters", WV_CHECK(wv_fill_u64((uint64_t*)md.rng_cnt, wv_cdiv(cells, 2), 0, s)));
    }
    WV_TIMED(prof, s, "tree_perm",
             WV_CHECK(wv_tree_permute(dlv, T, dseg, dtile, tile0.data(), digits ? &pc : nullptr, s)));
    uint8_t* dscr = p.h1 ? at<uint8_t>(ws, p.ws_sdir) : at<uint8_t>(ws, p.ws_wm + p.wm.off_dir);
    if (digits) {
        WV_TIMED(prof, s, "mcounters", WV_CHECK(wv_multiary_ranges(img, p.lay.lv, T, D, md, s)));
    } else if (shaped) {
        // level 0 is the longest
        WV_CHECK(wv_span_directory(img, p.lay, 0, K, dscr, wv_span_dir_sizes(p.lay.lv[0].n, K), s, prof));
    } else {
        WV_CHECK(wv_span_directory(img, p.lay, 0, K, dscr, p.wm.dir, s, prof));
    }
    // the host buffers copied from: pinned ones retire with the stream (the
    // call does not wait), pageable fallbacks must be waited for
    if (up_codes_v.size() || up_late_v.size()) {
        WV_CHECK(hipStreamSynchronize(s));
        up_codes.idle();
        late.idle();
    } else {
        up_codes.retire(s);
        late.retire(s);
    }
    return WT_OK;
}

int build_any(int kind, const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
              const wt_tuning* tune, void* out, size_t out_bytes, void* ws, size_t ws_bytes, hipStream_t s)
{
    Plan p;
    int rc = make_plan(kind, n, sigma, sym_bytes, shape, tune, p);
    if (rc) return rc;
    rc = check_buffers(p, S, out, out_bytes, ws, ws_bytes);
    if (rc) return rc;
    uint8_t* img = (uint8_t*)out;
    const bool prof = tune && (tune->flags & WT_FLAG_PROFILE);
    WV_TIMED(prof, s, "header", WV_CHECK(wv_write_header(img, p.lin, s)));
    if (p.from_matrix) return build_from_matrix(p, S, shape, img, (uint8_t*)ws, prof, s);

    if ((kind == WT_KIND_WM && !p.levelwise) || p.direct_tree) {
        // the first pass validates S while counting its digits
        wv_dir_scratch dir{at<uint32_t>(ws, p.ws_sb_ones), at<uint64_t>(ws, p.ws_sb_pre),
                           at<uint64_t>(ws, p.ws_partial), at<uint64_t>(ws, p.ws_scalars + 8)};
        WV_CHECK(wv_wm_run(p.wm, S, img, p.lay, at<uint8_t>(ws, p.ws_wm), dir, s));
        return WT_OK;
    }

    wv_lw_args a = lw_args(p, S, out, ws);
    a.profile = prof;
    if (is_tree(kind)) {
        uint64_t* dcounts = at<uint64_t>(ws, p.ws_counts);
        WV_CHECK(wv_validate(S, n, sym_bytes, sigma, img, dcounts, s));
        std::vector<uint64_t> counts(sigma);
        uint32_t status = 0;
        WV_CHECK(hipMemcpyAsync(counts.data(), dcounts, (uint64_t)sigma * 8, hipMemcpyDeviceToHost, s));
        WV_CHECK(hipMemcpyAsync(&status, img + 36, 4, hipMemcpyDeviceToHost, s));
        WV_CHECK(hipStreamSynchronize(s));
        if (status) return WT_ERANGE;
        HostNodes H;
        std::vector<uint8_t> rec;
        std::vector<uint8_t> code_rec;
        std::vector<uint32_t> c32, l32;
        if (kind == WT_KIND_SHAPED) {
            for (uint32_t x = 0; x < sigma; x++)
                if (counts[x] != shape->counts[x]) return WT_EINVAL;
            rc = shaped_nodes(*shape, sigma, H, rec);
            if (rc) return rc;
            code_rec.assign((uint64_t)sigma * WV_CODE_BYTES, 0);
            c32.resize(sigma);
            l32.resize(sigma);
            for (uint32_t x = 0; x < sigma; x++) {
                const uint64_t c = shape->code_len[x] ? shape->codes[x] : 0;
                const uint32_t len = shape->code_len[x];
                std::memcpy(code_rec.data() + (uint64_t)x * WV_CODE_BYTES, &c, 8);
                std::memcpy(code_rec.data() + (uint64_t)x * WV_CODE_BYTES + 8, &len, 4);
                c32[x] = (uint32_t)c;
                l32[x] = len;
            }
        } else {
            rc = balanced_nodes(counts, sigma, p.key_bits, p.D, p.nlevels, H);
            if (rc) return rc;
        }
        if (H.start.size() > p.node_bound) return WT_EUNSUP;
        WV_CHECK(hipMemcpyAsync((void*)a.nt.start, H.start.data(), H.start.size() * 4, hipMemcpyHostToDevice, s));
        WV_CHECK(hipMemcpyAsync((void*)a.nt.child_start, H.child_start.data(), H.child_start.size() * 4,
                                hipMemcpyHostToDevice, s));
        WV_CHECK(hipMemcpyAsync((void*)a.nt.child, H.child.data(), H.child.size() * 4, hipMemcpyHostToDevice, s));
        if (kind == WT_KIND_SHAPED) {
            WV_CHECK(hipMemcpyAsync((void*)a.codes, c32.data(), (uint64_t)sigma * 4, hipMemcpyHostToDevice, s));
            WV_CHECK(hipMemcpyAsync((void*)a.lens, l32.data(), (uint64_t)sigma * 4, hipMemcpyHostToDevice, s));
            if (!rec.empty())
                WV_CHECK(hipMemcpyAsync(img + p.lay.nodes_off, rec.data(), rec.size(), hipMemcpyHostToDevice, s));
            WV_CHECK(hipMemcpyAsync(img + p.lay.codes_off, code_rec.data(), code_rec.size(), hipMemcpyHostToDevice,
                                    s));
        }
        // the host vectors above go out of scope: finish the copies first
        WV_CHECK(hipStreamSynchronize(s));
    } else {
        WV_CHECK(wv_validate(S, n, sym_bytes, sigma, img, nullptr, s));
    }
    WV_CHECK(wv_run_levelwise(a, sym_bytes, s));
    return WT_OK;
}

}  // namespace

// ---- the allocation-free matrix build --------------------------------------
//
// Workspace of wm_build_noalloc: one array per device in the code object
// (placed by the loader, held until the process ends).  In host code the
// array's name is not a device address; its address on each device is looked
// up once per device, with that device current, and only that address is
// passed to kernels.
static __device__ __align__(256) uint8_t scratch[WT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;

// device address of `scratch` on the current device (nullptr on failure)
void* noalloc_scratch()
{
    static std::mutex mu;
    static void* ptr[NOALLOC_MAX_DEVICES] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        ptr[dev] = p;
    }
    return ptr[dev];
}

}  // namespace

hipStream_t wv_side_stream()
{
    static std::mutex mu;
    static std::vector<hipStream_t> streams;   // by device
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if (streams.size() <= (size_t)dev) streams.resize((size_t)dev + 1, nullptr);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) streams[dev] = nullptr;
    return streams[dev];
}

extern "C" {

const char* wt_strerror(int code)
{
    switch (code) {
    case WT_OK: return "ok";
    case WT_EINVAL: return "invalid argument";
    case WT_ERANGE: return "symbol out of range (>= sigma or without codeword)";
    case WT_ENOSPC: return "output or workspace buffer too small";
    case WT_EHIP: return "HIP runtime error";
    case WT_EUNSUP: return "outside the supported limits";
    default: return "unknown status";
    }
}

int wt_plan(int kind, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
            const wt_tuning* tune, wt_plan_info* info)
{
    if (!info) return WT_EINVAL;
    Plan p;
    int rc = make_plan(kind, n, sigma, sym_bytes, shape, tune, p);
    if (rc) return rc;
    std::memset(info, 0, sizeof(*info));
    info->kind = (uint32_t)kind;
    info->nlevels = p.nlevels;
    info->key_bits = p.key_bits;
    info->arity_log2 = p.lin.arity_log2;
    info->n = n;
    info->sigma = sigma;
    info->tau = p.tau;
    info->out_bytes = p.lay.image_bytes;
    info->workspace_bytes = p.ws_bytes;
    for (uint32_t l = 0; l < p.nlevels; l++) info->level_n[l] = p.lay.lv[l].n;
    info->split_bits = p.h1;
    info->split_long = p.nlong;
    return WT_OK;
}

int wt_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
             const wt_tuning* tune, void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream)
{
    const int kind = (shape && shape->codes) ? WT_KIND_SHAPED : WT_KIND_WT;
    return build_any(kind, S, n, sigma, sym_bytes, shape, tune, out, out_bytes, ws, ws_bytes, (hipStream_t)stream);
}

int wm_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
             const wt_tuning* tune, void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream)
{
    if (shape && (shape->codes || shape->arity_log2 > 1)) return WT_EINVAL;
    return build_any(WT_KIND_WM, S, n, sigma, sym_bytes, nullptr, tune, out, out_bytes, ws, ws_bytes,
                     (hipStream_t)stream);
}

int multiary_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_shape* shape,
                   const wt_tuning* tune, void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream)
{
    if (!shape || shape->codes) return WT_EINVAL;
    return build_any(WT_KIND_MULTIARY, S, n, sigma, sym_bytes, shape, tune, out, out_bytes, ws, ws_bytes,
                     (hipStream_t)stream);
}

int wm_build_noalloc(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_tuning* tune,
                     void* out, size_t out_bytes, void* stream)
{
    // per-kernel timing records events; this entry point takes no such option
    wt_tuning t = tune ? *tune : wt_tuning{};
    t.flags &= ~WT_FLAG_PROFILE;
    Plan p;
    int rc = make_plan(WT_KIND_WM, n, sigma, sym_bytes, nullptr, &t, p);
    if (rc) return rc;
    if (p.ws_bytes > WT_NOALLOC_SCRATCH_BYTES) return WT_ENOSPC;
    void* ws = noalloc_scratch();
    if (!ws) return WT_EHIP;
    return build_any(WT_KIND_WM, S, n, sigma, sym_bytes, nullptr, &t, out, out_bytes, ws, WT_NOALLOC_SCRATCH_BYTES,
                     (hipStream_t)stream);
}

int wt_check(const void* image, void* stream)
{
    if (!image) return WT_EINVAL;
    uint32_t status = 0;
    WV_CHECK(hipStreamSynchronize((hipStream_t)stream));
    WV_CHECK(hipMemcpy(&status, (const uint8_t*)image + 36, 4, hipMemcpyDeviceToHost));
    if (status & WV_STATUS_RANGE) return WT_ERANGE;
    return status ? WT_EINVAL : WT_OK;
}

int wt_image_bytes(const void* image, uint64_t* bytes, void* stream)
{
    if (!image || !bytes) return WT_EINVAL;
    uint32_t magic = 0;
    WV_CHECK(hipStreamSynchronize((hipStream_t)stream));
    WV_CHECK(hipMemcpy(&magic, image, 4, hipMemcpyDeviceToHost));
    if (magic != WV_MAGIC) return WT_EINVAL;
    WV_CHECK(hipMemcpy(bytes, (const uint8_t*)image + 40, 8, hipMemcpyDeviceToHost));
    return WT_OK;
}

int wt_symbol_counts(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma, uint64_t* counts, void* stream)
{
    if ((!S && n) || !counts || sigma == 0) return WT_EINVAL;
    if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4) return WT_EINVAL;
    WV_CHECK(wv_validate(S, n, sym_bytes, sigma, nullptr, counts, (hipStream_t)stream));
    return WT_OK;
}

// Canonical Huffman codewords.  Leaves are queued by (count, symbol); merged
// nodes are queued in creation order (their weights never decrease); each
// merge takes the two lightest heads, the leaf first on equal weight.
int wt_huffman_codes(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* code_len)
{
    if (!counts || !codes || !code_len) return WT_EINVAL;
    std::vector<std::pair<uint64_t, uint32_t>> leaves;
    for (uint32_t s = 0; s < sigma; s++) {
        codes[s] = 0;
        code_len[s] = 0;
        if (counts[s]) leaves.emplace_back(counts[s], s);
    }
    const size_t k = leaves.size();
    if (k == 0) return WT_OK;
    if (k == 1) {
        code_len[leaves[0].second] = 1;
        return WT_OK;
    }
    std::sort(leaves.begin(), leaves.end());
    // tree nodes: 0..k-1 leaves (sorted order), k.. merged nodes
    std::vector<uint64_t> merged_w;
    std::vector<size_t> up(2 * k - 1, 0);
    size_t lf = 0, mf = 0;
    while (merged_w.size() < k - 1) {
        size_t pick[2];
        uint64_t w = 0;
        for (int t = 0; t < 2; t++) {
            const bool leaf_ok = lf < k;
            const bool merged_ok = mf < merged_w.size();
            if (leaf_ok && (!merged_ok || leaves[lf].first <= merged_w[mf])) {
                w += leaves[lf].first;
                pick[t] = lf++;
            } else {
                w += merged_w[mf];
                pick[t] = k + mf++;
            }
        }
        const size_t id = k + merged_w.size();
        up[pick[0]] = up[pick[1]] = id;
        merged_w.push_back(w);
    }
    std::vector<uint32_t> depth(2 * k - 1, 0);
    for (size_t v = 2 * k - 2; v-- > 0;) depth[v] = depth[up[v]] + 1;
    std::vector<std::pair<uint32_t, uint32_t>> order;   // (length, symbol)
    for (size_t t = 0; t < k; t++) {
        if (depth[t] > 32) return WT_EUNSUP;
        code_len[leaves[t].second] = depth[t];
        order.emplace_back(depth[t], leaves[t].second);
    }
    std::sort(order.begin(), order.end());
    uint64_t c = 0;
    for (size_t t = 0; t < order.size(); t++) {
        if (t) c = (c + 1) << (order[t].first - order[t - 1].first);
        codes[order[t].second] = c;
    }
    return WT_OK;
}

}  // extern "C"
