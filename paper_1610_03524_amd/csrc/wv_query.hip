// wv_query.hip -- batched access / rank / select on built images.
//
// The queries are those of the problem statement (Sec. 2): access(i) = S[i],
// rank_c(i) = occurrences of c in S[0..i], select_c(k) = position of the k-th
// c.  They walk the levels without topology pointers (Sec. 2 notes the
// pointers can be dropped by changing the queries):
//   wavelet matrix: position i on level l maps to rank0(i) (bit 0) or
//     Z_l + rank1(i) (bit 1) on level l+1;
//   balanced trees: the node range [s, e) is refined by rank0 at s, i, e;
//   shaped trees: the node table gives every node's start and children;
//   multiary trees: per-digit counters replace rank0.
// select walks down to the symbol's range, then back up with select0/1,
// which takes the sub-sampled positions of ordinals 512j and 512(j+1) (the
// second sampling level of Clark's structure): a sub-range spanning 2^20 bits
// or more has every answer stored, any other is searched in the rank
// superblocks between the two (Sec. 5.1).  One thread answers one query.
#include "wv_internal.h"

namespace {

constexpr int Q_THREADS = 256;
constexpr uint64_t U64MAX = ~0ull;

struct QLevel {
    uint64_t n, zeros, bits_off, rank_off, sel0_off, sel1_off, nsel, sub_off, nsub, pool_off;
};

struct QImg {
    const uint8_t* img;
    uint32_t kind, D, nlevels, sigma;
    bool multi;   // levels of D-bit digits (multiary, or shaped over digits)
    uint64_t n, nodes_off, codes_off;
    QLevel lv[WV_MAX_LEVELS];
};

__device__ inline void load_image(const uint8_t* img, QImg& q)
{
    const uint32_t* h32 = (const uint32_t*)img;
    const uint64_t* h64 = (const uint64_t*)img;
    q.img = img;
    q.kind = h32[2];
    q.D = h32[3];
    q.n = h64[2];
    q.sigma = h32[6];
    q.nlevels = h32[7] > WV_MAX_LEVELS ? WV_MAX_LEVELS : h32[7];
    q.nodes_off = h64[7];
    q.codes_off = h64[9];
    q.multi = wv_multi_levels(q.kind, q.D);
    for (uint32_t l = 0; l < q.nlevels; l++) {
        const uint64_t* e = (const uint64_t*)(img + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * l);
        q.lv[l] = QLevel{e[0], e[1], e[3], e[4], e[5], e[6], e[7], 0, 0, 0};
        if (!q.multi) {   // binary: the sub-samples follow sel1, the pool them
            q.lv[l].sub_off = wv_sub_off(e[6], e[7]);
            q.lv[l].nsub = wv_nsub(e[0]);
            q.lv[l].pool_off = wv_pool_off(q.lv[l].sub_off, q.lv[l].nsub);
        }
    }
}

__device__ inline const uint64_t* words_of(const QImg& q, uint32_t l) { return (const uint64_t*)(q.img + q.lv[l].bits_off); }
__device__ inline const uint64_t* dir_of(const QImg& q, uint32_t l) { return (const uint64_t*)(q.img + q.lv[l].rank_off); }

__device__ inline uint32_t bit_at(const QImg& q, uint32_t l, uint64_t i)
{
    return (uint32_t)((words_of(q, l)[i >> 6] >> (i & 63)) & 1ull);
}

__device__ inline uint64_t rank0(const QImg& q, uint32_t l, uint64_t i) { return wv_rank0(words_of(q, l), dir_of(q, l), i); }
__device__ inline uint64_t rankb(const QImg& q, uint32_t l, uint32_t b, uint64_t i)
{
    const uint64_t z = rank0(q, l, i);
    return b ? i - z : z;
}

// position of the b-bit of 0-based ordinal j on level l (j < count of b-bits)
__device__ uint64_t selectb(const QImg& q, uint32_t l, uint32_t b, uint64_t j)
{
    const QLevel& L = q.lv[l];
    const uint32_t* sub = (const uint32_t*)(q.img + L.sub_off);
    // ordinals 512s and 512(s+1): ones from the front of the array, zeros
    // from its back; past the last one (zero) of the level the entry is n
    const uint64_t s = j / WV_SUB_STRIDE;
    const uint64_t p0 = b ? sub[s] : sub[L.nsub - 1 - s];
    const uint64_t p1 = b ? sub[s + 1] : sub[L.nsub - 2 - s];
    if (p1 - p0 >= (1ull << WV_XSPAN_LOG2)) {   // a long sub-range: the answer is stored
        const uint64_t nslot = wv_nslot(L.n);
        const uint32_t* pool = (const uint32_t*)(q.img + L.pool_off);
        return pool[((b ? 0 : nslot) + (p0 >> WV_XSPAN_LOG2)) * WV_SUB_STRIDE + (j % WV_SUB_STRIDE)];
    }
    return wv_select_dir(words_of(q, l), dir_of(q, l), L.n, b, j, p0, p1);
}

__device__ inline uint32_t digit_at(const QImg& q, uint32_t l, uint64_t i)
{
    const uint32_t P = 64u / q.D;
    return (uint32_t)((words_of(q, l)[i / P] >> (q.D * (i % P))) & ((1ull << q.D) - 1ull));
}

__device__ inline uint64_t mrank(const QImg& q, uint32_t l, uint32_t g, uint64_t i)
{
    return wv_mrank(words_of(q, l), q.img + q.lv[l].rank_off, q.lv[l].n, q.D, g, i);
}

struct QNode {
    uint64_t start, count;
    uint32_t level;
    const uint32_t* child;   // child[g] of the node's record
};

// node record k: binary {start, count, child[2], level, prefix}; D-bit
// digits {start, count, level, prefix, child[2^D]}
__device__ inline QNode node_at(const QImg& q, uint32_t k)
{
    const uint8_t* e = q.img + q.nodes_off + (uint64_t)k * wv_node_bytes(q.multi ? q.D : 1u);
    QNode nd;
    nd.start = ((const uint64_t*)e)[0];
    nd.count = ((const uint64_t*)e)[1];
    nd.level = ((const uint32_t*)e)[q.multi ? 4 : 6];
    nd.child = (const uint32_t*)e + (q.multi ? 6 : 4);
    return nd;
}

// a level's bit or digit at a position, its rank (occurrences of g in
// [0, i)) and its select (position of the g of 0-based ordinal j), for bit
// levels and digit levels alike (shaped trees)
__device__ inline uint32_t sym_at(const QImg& q, uint32_t l, uint64_t i)
{
    return q.multi ? digit_at(q, l, i) : bit_at(q, l, i);
}
__device__ inline uint64_t rank_sym_on(const QImg& q, uint32_t l, uint32_t g, uint64_t i)
{
    return q.multi ? mrank(q, l, g, i) : rankb(q, l, g, i);
}
__device__ inline uint64_t select_sym_on(const QImg& q, uint32_t l, uint32_t g, uint64_t j)
{
    if (!q.multi) return selectb(q, l, g, j);
    const QLevel& lv = q.lv[l];
    return wv_mselect(words_of(q, l), q.img + lv.rank_off, (const uint64_t*)(q.img + lv.sel0_off), lv.nsel, lv.n,
                      q.D, g, j);
}
// digit t (from the top) of a codeword of len digits
__device__ inline uint32_t code_digit(const QImg& q, uint64_t code, uint32_t len, uint32_t t)
{
    const uint32_t D = q.multi ? q.D : 1u;
    return (uint32_t)((code >> (D * (len - 1 - t))) & ((1ull << D) - 1ull));
}

// ---- access ------------------------------------------------------------------

__device__ uint32_t q_access(const QImg& q, uint64_t i)
{
    if (i >= q.n) return 0xFFFFFFFFu;
    uint32_t x = 0;
    if (q.kind == WT_KIND_WM) {
        for (uint32_t l = 0; l < q.nlevels; l++) {
            const uint32_t b = bit_at(q, l, i);
            const uint64_t z = rank0(q, l, i);
            i = b ? q.lv[l].zeros + (i - z) : z;
            x = (x << 1) | b;
        }
        return x;
    }
    if (q.kind == WT_KIND_WT) {
        uint64_t s = 0, e = q.n;
        for (uint32_t l = 0; l < q.nlevels; l++) {
            const uint32_t b = bit_at(q, l, i);
            const uint64_t zs = rank0(q, l, s), zi = rank0(q, l, i), ze = rank0(q, l, e);
            if (!b) {
                i = s + (zi - zs);
                e = s + (ze - zs);
            } else {
                i = s + (ze - zs) + (i - s) - (zi - zs);
                s = s + (ze - zs);
            }
            x = (x << 1) | b;
        }
        return x;
    }
    if (q.kind == WT_KIND_MULTIARY) {
        uint64_t s = 0, e = q.n;
        const uint32_t d = 1u << q.D;
        for (uint32_t l = 0; l < q.nlevels; l++) {
            const uint32_t g = digit_at(q, l, i);
            uint64_t below = 0;
            for (uint32_t c = 0; c < g; c++) below += mrank(q, l, c, e) - mrank(q, l, c, s);
            const uint64_t gs = mrank(q, l, g, s);
            const uint64_t cs = s + below;
            const uint64_t ni = cs + mrank(q, l, g, i) - gs;
            e = cs + mrank(q, l, g, e) - gs;
            s = cs;
            i = ni;
            x = (x << q.D) | g;
            (void)d;
        }
        return x;
    }
    // shaped: follow the node table
    uint32_t k = 0;
    uint64_t rel = i;
    for (uint32_t step = 0; step <= WV_MAX_LEVELS; step++) {
        const QNode nd = node_at(q, k);
        const uint64_t pos = nd.start + rel;
        const uint32_t b = sym_at(q, nd.level, pos);
        rel = rank_sym_on(q, nd.level, b, pos) - rank_sym_on(q, nd.level, b, nd.start);
        const uint32_t c = nd.child[b];
        if (c & WV_LEAF) return c == WV_NONE ? 0xFFFFFFFFu : (c & ~WV_LEAF);
        k = c;
    }
    return 0xFFFFFFFFu;
}

// ---- rank / select ---------------------------------------------------------------

__device__ inline bool shaped_code(const QImg& q, uint32_t c, uint64_t& code, uint32_t& len)
{
    if (c >= q.sigma) return false;
    const uint8_t* e = q.img + q.codes_off + (uint64_t)c * WV_CODE_BYTES;
    code = ((const uint64_t*)e)[0];
    len = ((const uint32_t*)e)[2];
    return len != 0;
}

// occurrences of c among the first p symbols (positions 0..p-1)
__device__ uint64_t q_count_prefix(const QImg& q, uint32_t c, uint64_t p)
{
    const uint32_t L = q.nlevels;
    if (q.kind == WT_KIND_WM) {
        uint64_t s = 0, e = p;
        for (uint32_t l = 0; l < L; l++) {
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            const uint64_t zs = rank0(q, l, s), ze = rank0(q, l, e);
            if (b) { s = q.lv[l].zeros + s - zs; e = q.lv[l].zeros + e - ze; }
            else { s = zs; e = ze; }
        }
        return e - s;
    }
    if (q.kind == WT_KIND_WT) {
        uint64_t s = 0, e = q.n;
        for (uint32_t l = 0; l < L; l++) {
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            const uint64_t zs = rank0(q, l, s), zp = rank0(q, l, p), ze = rank0(q, l, e);
            if (!b) {
                p = s + (zp - zs);
                e = s + (ze - zs);
            } else {
                p = s + (ze - zs) + (p - s) - (zp - zs);
                s = s + (ze - zs);
            }
        }
        return p - s;
    }
    if (q.kind == WT_KIND_MULTIARY) {
        uint64_t s = 0, e = q.n;
        for (uint32_t l = 0; l < L; l++) {
            const uint32_t g = (c >> (q.D * (L - 1 - l))) & ((1u << q.D) - 1u);
            uint64_t below = 0;
            for (uint32_t cc = 0; cc < g; cc++) below += mrank(q, l, cc, e) - mrank(q, l, cc, s);
            const uint64_t gs = mrank(q, l, g, s);
            const uint64_t cs = s + below;
            p = cs + mrank(q, l, g, p) - gs;
            e = cs + mrank(q, l, g, e) - gs;
            s = cs;
        }
        return p - s;
    }
    uint64_t code;
    uint32_t len;
    if (!shaped_code(q, c, code, len)) return 0;
    uint32_t k = 0;
    uint64_t rel = p;
    for (uint32_t t = 0; t < len; t++) {
        const QNode nd = node_at(q, k);
        const uint32_t b = code_digit(q, code, len, t);
        const uint64_t pos = nd.start + rel;
        rel = rank_sym_on(q, nd.level, b, pos) - rank_sym_on(q, nd.level, b, nd.start);
        k = nd.child[b];
    }
    return rel;
}

__device__ uint64_t q_rank(const QImg& q, uint32_t c, uint64_t i)
{
    if (i >= q.n) return U64MAX;
    if (c >= q.sigma) return 0;
    return q_count_prefix(q, c, i + 1);
}

__device__ uint64_t q_select(const QImg& q, uint32_t c, uint64_t k)
{
    if (k == 0 || c >= q.sigma || q.n == 0) return U64MAX;
    const uint32_t L = q.nlevels;
    // matrix and balanced tree: one descent gives the symbol's range [s, e)
    // below the last level, so its length is the symbol's count
    if (q.kind == WT_KIND_WM) {
        uint64_t s = 0, e = q.n;
        for (uint32_t l = 0; l < L; l++) {
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            const uint64_t zs = rank0(q, l, s), ze = rank0(q, l, e);
            if (b) { s = q.lv[l].zeros + s - zs; e = q.lv[l].zeros + e - ze; }
            else { s = zs; e = ze; }
        }
        if (k > e - s) return U64MAX;
        uint64_t p = s + k - 1;
        for (uint32_t l = L; l-- > 0;) {
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            p = selectb(q, l, b, b ? p - q.lv[l].zeros : p);
        }
        return p;
    }
    if (q.kind == WT_KIND_WT) {
        uint64_t starts[WV_MAX_LEVELS];
        uint64_t s = 0, e = q.n;
        for (uint32_t l = 0; l < L; l++) {
            starts[l] = s;
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            const uint64_t zs = rank0(q, l, s), ze = rank0(q, l, e);
            if (!b) e = s + (ze - zs); else s = s + (ze - zs);
        }
        if (k > e - s) return U64MAX;
        uint64_t p = s + k - 1, child = s;
        for (uint32_t l = L; l-- > 0;) {
            const uint32_t b = (c >> (L - 1 - l)) & 1u;
            const uint64_t st = starts[l];
            p = selectb(q, l, b, rankb(q, l, b, st) + (p - child));
            child = st;
        }
        return p;
    }
    const uint64_t total = q_count_prefix(q, c, q.n);
    if (k > total) return U64MAX;
    if (q.kind == WT_KIND_SHAPED) {
        uint64_t code;
        uint32_t len;
        shaped_code(q, c, code, len);
        uint32_t path[WV_MAX_LEVELS];
        uint32_t kk = 0;
        for (uint32_t t = 0; t < len; t++) {
            path[t] = kk;
            kk = node_at(q, kk).child[code_digit(q, code, len, t)];
        }
        uint64_t rel = k - 1;
        for (uint32_t t = len; t-- > 0;) {
            const QNode nd = node_at(q, path[t]);
            const uint32_t b = code_digit(q, code, len, t);
            rel = select_sym_on(q, nd.level, b, rank_sym_on(q, nd.level, b, nd.start) + rel) - nd.start;
        }
        return rel;
    }
    // multiary: the descent gives c's node start on every level; walking up,
    // the rel-th symbol of a child node is the (rel+1)-th digit of its value
    // in the parent node: a generalized select on that level (Sec. 5.2)
    uint64_t starts[WV_MAX_LEVELS];
    uint64_t s = 0, e = q.n;
    for (uint32_t l = 0; l < L; l++) {
        starts[l] = s;
        const uint32_t g = (c >> (q.D * (L - 1 - l))) & ((1u << q.D) - 1u);
        uint64_t below = 0;
        for (uint32_t cc = 0; cc < g; cc++) below += mrank(q, l, cc, e) - mrank(q, l, cc, s);
        const uint64_t gs = mrank(q, l, g, s);
        const uint64_t cs = s + below;
        e = cs + mrank(q, l, g, e) - gs;
        s = cs;
    }
    uint64_t rel = k - 1;
    for (uint32_t l = L; l-- > 0;) {
        const uint32_t g = (c >> (q.D * (L - 1 - l))) & ((1u << q.D) - 1u);
        const uint64_t st = starts[l];
        const QLevel& lv = q.lv[l];
        rel = wv_mselect(words_of(q, l), q.img + lv.rank_off, (const uint64_t*)(q.img + lv.sel0_off), lv.nsel, lv.n,
                         q.D, g, mrank(q, l, g, st) + rel) - st;
    }
    return rel;
}

__global__ void __launch_bounds__(Q_THREADS)
access_k(const uint8_t* __restrict__ img, const uint64_t* __restrict__ pos, uint32_t* __restrict__ res, uint64_t m)
{
    __shared__ QImg q;
    if (threadIdx.x == 0) load_image(img, q);
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * Q_THREADS + threadIdx.x;
    if (t < m) res[t] = q_access(q, pos[t]);
}

__global__ void __launch_bounds__(Q_THREADS)
rank_k(const uint8_t* __restrict__ img, const uint32_t* __restrict__ c, const uint64_t* __restrict__ i,
       uint64_t* __restrict__ res, uint64_t m)
{
    __shared__ QImg q;
    if (threadIdx.x == 0) load_image(img, q);
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * Q_THREADS + threadIdx.x;
    if (t < m) res[t] = q_rank(q, c[t], i[t]);
}

__global__ void __launch_bounds__(Q_THREADS)
select_k(const uint8_t* __restrict__ img, const uint32_t* __restrict__ c, const uint64_t* __restrict__ k,
         uint64_t* __restrict__ res, uint64_t m)
{
    __shared__ QImg q;
    if (threadIdx.x == 0) load_image(img, q);
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * Q_THREADS + threadIdx.x;
    if (t < m) res[t] = q_select(q, c[t], k[t]);
}

}  // namespace

extern "C" {

int wt_access(const void* image, const uint64_t* pos, uint32_t* res, uint64_t m, void* stream)
{
    if (!image || (m && (!pos || !res))) return WT_EINVAL;
    if (!m) return WT_OK;
    if (wv_cdiv(m, Q_THREADS) > 0x7FFFFFFFull) return WT_EUNSUP;   // one thread a query, grid.x < 2^31
    access_k<<<(uint32_t)wv_cdiv(m, Q_THREADS), Q_THREADS, 0, (hipStream_t)stream>>>(
        (const uint8_t*)image, pos, res, m);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_EHIP;
}

int wt_rank(const void* image, const uint32_t* c, const uint64_t* i, uint64_t* res, uint64_t m, void* stream)
{
    if (!image || (m && (!c || !i || !res))) return WT_EINVAL;
    if (!m) return WT_OK;
    if (wv_cdiv(m, Q_THREADS) > 0x7FFFFFFFull) return WT_EUNSUP;   // one thread a query, grid.x < 2^31
    rank_k<<<(uint32_t)wv_cdiv(m, Q_THREADS), Q_THREADS, 0, (hipStream_t)stream>>>(
        (const uint8_t*)image, c, i, res, m);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_EHIP;
}

int wt_select(const void* image, const uint32_t* c, const uint64_t* k, uint64_t* res, uint64_t m, void* stream)
{
    if (!image || (m && (!c || !k || !res))) return WT_EINVAL;
    if (!m) return WT_OK;
    if (wv_cdiv(m, Q_THREADS) > 0x7FFFFFFFull) return WT_EUNSUP;   // one thread a query, grid.x < 2^31
    select_k<<<(uint32_t)wv_cdiv(m, Q_THREADS), Q_THREADS, 0, (hipStream_t)stream>>>(
        (const uint8_t*)image, c, k, res, m);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_EHIP;
}

}  // extern "C"
