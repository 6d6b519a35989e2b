/*
 * wavelet_oracle.c -- plain, slow, level-by-level CPU reference builder.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the GPU library: every layout rule
 * used here is written out again from its definition.
 *
 * What it computes (Shun, "Improved Parallel Construction of Wavelet Trees
 * and Rank/Select Structures"):
 *   - the balanced binary wavelet tree, levelwise and pointerless
 *     (Sec. 2: recursive definition of the tree over [0, 2^ceil(log sigma)-1];
 *      the topology pointers are dropped, as Sec. 2 notes is possible);
 *   - the wavelet matrix (Sec. 4.3, paragraph "Wavelet matrix");
 *   - the arbitrary-shaped binary wavelet tree given codewords
 *     (Sec. 4.3, paragraph "Arbitrarily-shaped binary trees"), and the same
 *     over codewords of D-bit digits, a shaped multiary tree (the paper notes
 *     shapes carry over to multiary trees);
 *   - the balanced multiary wavelet tree of degree d = 2^D
 *     (Sec. 4.3, paragraph "Multiary wavelet trees");
 *   - the rank-of-0 directory of every binary level (Sec. 5.1, "Rank":
 *     Jacobson's ranges and sub-ranges, here 512-bit ranges and 64-bit
 *     sub-ranges) and sampled select (Sec. 5.1, "Select": the two sampling
 *     levels of Clark's structure, here every 4096th and every 512th one and
 *     zero, plus Clark's rule of storing every answer of a long range, here
 *     for the 512-one sub-ranges spanning 2^20 bits or more);
 *   - per-digit rank counters on multiary levels (Sec. 5.2, "Rank") and
 *     per-digit sampled select (Sec. 5.2, "Select": the range symbols, every
 *     4096th occurrence of each digit value);
 *   - canonical Huffman codewords, the shape used for Huffman-shaped trees.
 *
 * Every structure is a deterministic function of (S, sigma, kind, shape);
 * the output is one flat byte image whose layout is fixed below.
 *
 * Pins (tests that check this file against something other than itself):
 * the hand-derived example on the sequence of Fig. 1, brute-force queries
 * walked through the image on all tiny inputs, closed forms by stable
 * argsort, cumulative-sum directories, Huffman optimality and Kraft sums.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- status codes returned to the caller -------------------------------- */
#define O_OK      0
#define O_EINVAL  (-1)
#define O_ERANGE  (-2)
#define O_ENOMEM  (-3)
#define O_EUNSUP  (-5)

/* ---- structure kinds ---------------------------------------------------- */
#define O_KIND_WT      1   /* balanced binary wavelet tree */
#define O_KIND_WM      2   /* wavelet matrix */
#define O_KIND_SHAPED  3   /* binary wavelet tree shaped by given codewords */
#define O_KIND_MULTI   4   /* balanced multiary wavelet tree, d = 2^D */

/* ---- image layout ------------------------------------------------------- */
#define O_MAGIC        0x54564157u  /* bytes 'W','A','V','T' */
#define O_VERSION      3u
#define O_HEADER_BYTES 256u
#define O_LEVEL_BYTES  64u
#define O_NODE_BYTES   32u    /* binary shaped trees */
/* shaped trees of D-bit digits (D >= 2): u64 start, u64 count, u32 level,
 * u32 prefix, u32 child[2^D] */
static uint64_t mnode_bytes(unsigned D) { return 24u + 4u * ((uint64_t)1 << D); }
static uint64_t node_bytes(unsigned D) { return D >= 2 ? mnode_bytes(D) : O_NODE_BYTES; }
#define O_CODE_BYTES   16u
#define O_RANGE_BITS   512u   /* rank directory range (superblock) */
#define O_SUB_BITS     64u    /* rank directory sub-range (block) */
#define O_SEL_STRIDE   4096u  /* select sampling stride */
#define O_SUB_STRIDE   512u   /* select sub-sampling stride (second level) */
#define O_LONG_SPAN    (1ull << 20)  /* a sub-range this long keeps every answer */
#define O_LEAF_FLAG    0x80000000u
#define O_NO_CHILD     0xFFFFFFFFu
#define O_MAX_CODE_LEN 32u

typedef struct {
    uint64_t n;         /* bits (binary) or digits (multiary) on the level */
    uint64_t zeros;     /* binary: number of 0 bits */
    uint64_t ones;      /* binary: number of 1 bits */
    uint64_t bits_off;  /* packed words */
    uint64_t rank_off;  /* rank directory / digit counters */
    uint64_t sel0_off;  /* sampled select on zeros */
    uint64_t sel1_off;  /* sampled select on ones */
    uint64_t nsel;      /* entries in each sampled-select array */
    uint64_t sub_off;   /* binary: select sub-samples, ones from the front,
                           zeros from the back (32-bit positions) */
    uint64_t nsub;      /* entries of the sub-sample array */
    uint64_t pool_off;  /* binary: stored answers of long sub-ranges */
    uint64_t nslot;     /* slots of 512 answers per kind (ones, then zeros) */
} olevel;

static uint64_t round256(uint64_t x) { return (x + 255u) & ~(uint64_t)255u; }
static uint64_t min_u64(uint64_t a, uint64_t b) { return a < b ? a : b; }

static void put_u32(uint8_t* p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }
static void put_u16(uint8_t* p, uint16_t v) { memcpy(p, &v, 2); }

/* L = max(1, ceil(log2 sigma)): the root covers [0, 2^L - 1] (Sec. 2). */
static unsigned key_bits_of(uint32_t sigma)
{
    unsigned L = 1;
    while (L < 32 && ((uint64_t)1 << L) < sigma) L++;
    return L;
}

/* Digits packed into one 64-bit word for D-bit digits. */
static unsigned digits_per_word(unsigned D) { return 64u / D; }

/* Sizes of the arrays of one binary level holding m bits. */
static uint64_t bin_bits_bytes(uint64_t m) { return ((m + 63) / 64) * 8; }
static uint64_t bin_rank_bytes(uint64_t m)
{
    return ((m + O_RANGE_BITS - 1) / O_RANGE_BITS + 1) * 16;
}
static uint64_t bin_nsel(uint64_t m) { return (m + O_SEL_STRIDE - 1) / O_SEL_STRIDE + 1; }
/* ceil(ones/512) + ceil(zeros/512) <= ceil(m/512) + 1 entries are used, so
 * one more leaves at least one unused entry between the two halves */
static uint64_t bin_nsub(uint64_t m) { return (m + O_SUB_STRIDE - 1) / O_SUB_STRIDE + 2; }

/* Sizes for one multiary level of m digits of D bits. */
static uint64_t multi_bits_bytes(uint64_t m, unsigned D)
{
    uint64_t p = digits_per_word(D);
    return ((m + p - 1) / p) * 8;
}
static uint64_t multi_rank_bytes(uint64_t m, unsigned D)
{
    uint64_t p = digits_per_word(D), d = (uint64_t)1 << D;
    uint64_t sbd = 64 * p, bd = 8 * p;
    uint64_t nsb = (m + sbd - 1) / sbd, nb = (m + bd - 1) / bd;
    return (nsb + 1) * d * 8 + nb * d * 2;
}

/* Assign the offsets of every array.  Binary levels hold bits, rank, sel0,
 * sel1 and the select sub-samples; multiary levels hold digits, counters and
 * per-digit samples; shaped trees append the node table and the code table.
 * Every array starts on a 256-byte boundary. */
static uint64_t lay_out(olevel* lv, unsigned nlev, int multiary, unsigned D,
                        uint64_t nnodes, uint32_t sigma, int shaped,
                        uint64_t* nodes_off, uint64_t* codes_off)
{
    uint64_t off = O_HEADER_BYTES + round256((uint64_t)O_LEVEL_BYTES * nlev);
    for (unsigned l = 0; l < nlev; l++) {
        uint64_t m = lv[l].n;
        lv[l].bits_off = off;
        off = round256(off + (multiary ? multi_bits_bytes(m, D) : bin_bits_bytes(m)));
        lv[l].rank_off = off;
        off = round256(off + (multiary ? multi_rank_bytes(m, D) : bin_rank_bytes(m)));
        if (!multiary) {
            lv[l].nsel = bin_nsel(m);
            lv[l].sel0_off = off;
            off = round256(off + lv[l].nsel * 8);
            lv[l].sel1_off = off;
            off = round256(off + lv[l].nsel * 8);
            lv[l].nsub = bin_nsub(m);
            lv[l].sub_off = off;
            off = round256(off + lv[l].nsub * 4);
            /* long sub-ranges are disjoint and at least 2^20 bits each, so
             * a level of m bits has at most floor(m / 2^20) of each kind */
            lv[l].nslot = m / O_LONG_SPAN;
            lv[l].pool_off = off;
            off = round256(off + lv[l].nslot * 2 * O_SUB_STRIDE * 4);
        } else {
            /* generalized select: d arrays of nsel samples, digit-major */
            lv[l].nsel = bin_nsel(m);
            lv[l].sel0_off = off;
            off = round256(off + ((uint64_t)1 << D) * lv[l].nsel * 8);
            lv[l].sel1_off = 0;
            lv[l].sub_off = lv[l].nsub = 0;
            lv[l].pool_off = lv[l].nslot = 0;
        }
    }
    *nodes_off = *codes_off = 0;
    if (shaped) {
        *nodes_off = off;
        off = round256(off + nnodes * node_bytes(D));
        *codes_off = off;
        off = round256(off + (uint64_t)sigma * O_CODE_BYTES);
    }
    return off;
}

/* Write one binary level: bits b[0..m) packed LSB-first, its rank-of-0
 * directory and its sampled select arrays (Sec. 5.1).  The rank directory
 * holds, for every range k = 0..ceil(m/512), the zeros before the range
 * (the exclusive prefix sum of per-word zero counts of Sec. 5.1, read at
 * every range boundary) and seven 9-bit counts of zeros from the range start
 * to each later 64-bit sub-range boundary (the relative sub-range counts). */
static int write_binary_level(uint8_t* img, olevel* lv, const uint8_t* b)
{
    uint64_t m = lv->n;
    uint64_t* zp = (uint64_t*)malloc((m + 1) * sizeof(uint64_t));
    if (!zp) return O_ENOMEM;
    uint8_t* words = img + lv->bits_off;
    zp[0] = 0;
    for (uint64_t i = 0; i < m; i++) {
        zp[i + 1] = zp[i] + (b[i] == 0);
        if (b[i]) words[i >> 3] |= (uint8_t)(1u << (i & 7));  /* LSB-first */
    }
    lv->zeros = zp[m];
    lv->ones = m - zp[m];

    uint64_t nranges = (m + O_RANGE_BITS - 1) / O_RANGE_BITS;
    uint8_t* r = img + lv->rank_off;
    for (uint64_t k = 0; k <= nranges; k++) {
        uint64_t s = k * O_RANGE_BITS;
        uint64_t abs0 = zp[min_u64(s, m)];
        uint64_t rel = 0;
        if (s < m) {
            for (unsigned j = 1; j <= 7; j++) {
                uint64_t hi = min_u64(s + (uint64_t)O_SUB_BITS * j, m);
                rel |= (zp[hi] - zp[s]) << (9 * (j - 1));
            }
        }
        put_u64(r + 16 * k, abs0);
        put_u64(r + 16 * k + 8, rel);
    }

    /* Sampled select: position of the one (zero) whose 0-based ordinal is a
     * multiple of 4096; unused entries hold m. */
    uint8_t* s0 = img + lv->sel0_off;
    uint8_t* s1 = img + lv->sel1_off;
    for (uint64_t k = 0; k < lv->nsel; k++) {
        put_u64(s0 + 8 * k, m);
        put_u64(s1 + 8 * k, m);
    }
    /* Second sampling level of Clark's structure (Sec. 5.1, "Select"): the
     * position of every one (zero) whose ordinal is a multiple of 512, so a
     * select only searches the rank ranges between two such positions.  As
     * n < 2^32 the positions themselves fit 32 bits (no offsets relative to
     * the first level are needed).  Ones fill the array from the front, zeros
     * from the back (entry nsub-1-j holds zero 512j); entries left between
     * the two hold m. */
    uint8_t* sub = img + lv->sub_off;
    for (uint64_t k = 0; k < lv->nsub; k++) put_u32(sub + 4 * k, (uint32_t)m);
    uint64_t c0 = 0, c1 = 0;
    for (uint64_t i = 0; i < m; i++) {
        if (b[i]) {
            if (c1 % O_SEL_STRIDE == 0) put_u64(s1 + 8 * (c1 / O_SEL_STRIDE), i);
            if (c1 % O_SUB_STRIDE == 0) put_u32(sub + 4 * (c1 / O_SUB_STRIDE), (uint32_t)i);
            c1++;
        } else {
            if (c0 % O_SEL_STRIDE == 0) put_u64(s0 + 8 * (c0 / O_SEL_STRIDE), i);
            if (c0 % O_SUB_STRIDE == 0) put_u32(sub + 4 * (lv->nsub - 1 - c0 / O_SUB_STRIDE), (uint32_t)i);
            c0++;
        }
    }
    /* Clark's rule for long ranges (Sec. 5.1, "Select"): when the stretch
     * from the one (zero) of ordinal 512j to that of ordinal 512(j+1) (to m
     * if there is none) is at least 2^20 bits, every answer in it is stored:
     * the positions of ordinals 512j, 512j+1, ... (at most 512 of them) in
     * slot floor(p / 2^20) of the kind's pool, p being the stretch's start.
     * The pool holds the ones' slots, then the zeros'; unused entries m. */
    if (lv->nslot) {
        uint8_t* pool = img + lv->pool_off;
        for (uint64_t k = 0; k < 2 * lv->nslot * O_SUB_STRIDE; k++) put_u32(pool + 4 * k, (uint32_t)m);
        uint64_t* pos = (uint64_t*)malloc((m + 1) * sizeof(uint64_t));
        if (!pos) { free(zp); return O_ENOMEM; }
        for (int kind = 1; kind >= 0; kind--) {
            uint64_t cnt = 0;   /* positions of this kind's bits, in order */
            for (uint64_t i = 0; i < m; i++)
                if ((b[i] != 0) == (kind == 1)) pos[cnt++] = i;
            for (uint64_t j0 = 0; j0 < cnt; j0 += O_SUB_STRIDE) {
                uint64_t start = pos[j0];
                uint64_t end = j0 + O_SUB_STRIDE < cnt ? pos[j0 + O_SUB_STRIDE] : m;
                if (end - start < O_LONG_SPAN) continue;
                uint64_t slot = (kind == 1 ? 0 : lv->nslot) + start / O_LONG_SPAN;
                for (uint64_t t = 0; t < O_SUB_STRIDE && j0 + t < cnt; t++)
                    put_u32(pool + 4 * (slot * O_SUB_STRIDE + t), (uint32_t)pos[j0 + t]);
            }
        }
        free(pos);
    }
    free(zp);
    return O_OK;
}

/* Write one multiary level: digits g[0..m) of D bits, packed floor(64/D) per
 * word (digit t at bits [tD, tD+D) of its word), followed by its per-digit
 * rank counters (Sec. 5.2, "Rank"): for every range of 64 words the count of
 * each digit before the range, and for every sub-range of 8 words the count
 * of each digit from the start of its range to the start of the sub-range. */
static void write_multi_level(uint8_t* img, olevel* lv, const uint8_t* g, unsigned D)
{
    uint64_t m = lv->n, p = digits_per_word(D), d = (uint64_t)1 << D;
    uint64_t sbd = 64 * p, bd = 8 * p;
    uint64_t nsb = (m + sbd - 1) / sbd;
    uint8_t* words = img + lv->bits_off;
    for (uint64_t t = 0; t < m; t++) {
        uint64_t w;
        memcpy(&w, words + 8 * (t / p), 8);
        w |= (uint64_t)g[t] << (D * (t % p));
        memcpy(words + 8 * (t / p), &w, 8);
    }
    uint8_t* sb = img + lv->rank_off;
    uint8_t* blk = sb + (nsb + 1) * d * 8;
    uint64_t cnt[16] = {0};
    uint64_t at_range[16] = {0};
    for (uint64_t t = 0; t < m; t++) {
        if (t % sbd == 0) {
            for (uint64_t c = 0; c < d; c++) {
                put_u64(sb + ((t / sbd) * d + c) * 8, cnt[c]);
                at_range[c] = cnt[c];
            }
        }
        if (t % bd == 0) {
            for (uint64_t c = 0; c < d; c++)
                put_u16(blk + ((t / bd) * d + c) * 2, (uint16_t)(cnt[c] - at_range[c]));
        }
        cnt[g[t]]++;
    }
    /* the sentinel range entry k = nsb holds the totals */
    for (uint64_t c = 0; c < d; c++) put_u64(sb + (nsb * d + c) * 8, cnt[c]);
    /* Generalized select (Sec. 5.2, "Select"): a separate sampled structure
       for every character, here every digit value c: the position of the
       occurrence of c whose 0-based ordinal is 4096k (the range symbols of
       c), then m in the entries past the last one */
    uint8_t* sel = img + lv->sel0_off;
    uint64_t seen[16] = {0};
    for (uint64_t c = 0; c < d; c++)
        for (uint64_t k = 0; k < lv->nsel; k++) put_u64(sel + (c * lv->nsel + k) * 8, m);
    for (uint64_t t = 0; t < m; t++) {
        uint64_t c = g[t];
        if (seen[c] % O_SEL_STRIDE == 0) put_u64(sel + (c * lv->nsel + seen[c] / O_SEL_STRIDE) * 8, t);
        seen[c]++;
    }
}

static void write_header(uint8_t* img, int kind, unsigned arity_log2, uint64_t n,
                         uint32_t sigma, unsigned nlev, unsigned key_bits,
                         uint64_t image_bytes, uint64_t nodes_off, uint64_t nnodes,
                         uint64_t codes_off, uint64_t ncoded, const olevel* lv)
{
    put_u32(img + 0, O_MAGIC);
    put_u32(img + 4, O_VERSION);
    put_u32(img + 8, (uint32_t)kind);
    put_u32(img + 12, arity_log2);
    put_u64(img + 16, n);
    put_u32(img + 24, sigma);
    put_u32(img + 28, nlev);
    put_u32(img + 32, key_bits);
    put_u32(img + 36, 0);            /* status: 0 = every symbol < sigma */
    put_u64(img + 40, image_bytes);
    put_u64(img + 48, O_HEADER_BYTES);
    put_u64(img + 56, nodes_off);
    put_u64(img + 64, nnodes);
    put_u64(img + 72, codes_off);
    put_u64(img + 80, ncoded);
    for (unsigned l = 0; l < nlev; l++) {
        uint8_t* e = img + O_HEADER_BYTES + (uint64_t)O_LEVEL_BYTES * l;
        put_u64(e + 0, lv[l].n);
        put_u64(e + 8, lv[l].zeros);
        put_u64(e + 16, lv[l].ones);
        put_u64(e + 24, lv[l].bits_off);
        put_u64(e + 32, lv[l].rank_off);
        put_u64(e + 40, lv[l].sel0_off);
        put_u64(e + 48, lv[l].sel1_off);
        put_u64(e + 56, lv[l].nsel);
    }
}

static int read_symbols(const void* S, int sym_bytes, uint64_t n, uint32_t sigma,
                        uint32_t** out)
{
    if (sym_bytes != 1 && sym_bytes != 2 && sym_bytes != 4) return O_EINVAL;
    uint32_t* x = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    if (!x) return O_ENOMEM;
    for (uint64_t i = 0; i < n; i++) {
        if (sym_bytes == 1) x[i] = ((const uint8_t*)S)[i];
        else if (sym_bytes == 2) x[i] = ((const uint16_t*)S)[i];
        else x[i] = ((const uint32_t*)S)[i];
        if (x[i] >= sigma) { free(x); return O_ERANGE; }
    }
    *out = x;
    return O_OK;
}

/* Balanced binary tree, levelwise (Sec. 2).  Level l concatenates the node
 * bitstrings of depth l in left-to-right node order.  A node at depth l holds
 * the symbols sharing their top l bits, in input order; its bit for a symbol
 * is bit l from the top (0 = left half of the node's range).  Going down one
 * level stably partitions every node by that bit. */
static int build_wt(uint8_t* img, olevel* lv, unsigned L, uint32_t* cur, uint64_t n)
{
    uint32_t* nxt = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    uint8_t* b = (uint8_t*)malloc(n ? n : 1);
    if (!nxt || !b) { free(nxt); free(b); return O_ENOMEM; }
    for (unsigned l = 0; l < L; l++) {
        unsigned sh = L - 1 - l;
        for (uint64_t i = 0; i < n; i++) b[i] = (uint8_t)(((uint64_t)cur[i] >> sh) & 1);
        int rc = write_binary_level(img, &lv[l], b);
        if (rc) { free(nxt); free(b); return rc; }
        /* stable partition inside each node: nodes are the maximal runs of
         * equal top-l-bit prefix */
        uint64_t s = 0;
        while (s < n) {
            uint64_t e = s + 1;
            if (l > 0) {
                uint64_t p = (uint64_t)cur[s] >> (L - l);
                while (e < n && ((uint64_t)cur[e] >> (L - l)) == p) e++;
            } else {
                e = n;
            }
            uint64_t o = s;
            for (uint64_t i = s; i < e; i++) if (!b[i]) nxt[o++] = cur[i];
            for (uint64_t i = s; i < e; i++) if (b[i]) nxt[o++] = cur[i];
            s = e;
        }
        memcpy(cur, nxt, n * sizeof(uint32_t));
    }
    free(nxt);
    free(b);
    return O_OK;
}

/* Wavelet matrix (Sec. 4.3): level l holds bit l from the top of every symbol;
 * the next level puts the symbols with a 0 there first and those with a 1
 * after them, each side in the order of the current level. */
static int build_wm(uint8_t* img, olevel* lv, unsigned L, uint32_t* cur, uint64_t n)
{
    uint32_t* nxt = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    uint8_t* b = (uint8_t*)malloc(n ? n : 1);
    if (!nxt || !b) { free(nxt); free(b); return O_ENOMEM; }
    for (unsigned l = 0; l < L; l++) {
        unsigned sh = L - 1 - l;
        for (uint64_t i = 0; i < n; i++) b[i] = (uint8_t)(((uint64_t)cur[i] >> sh) & 1);
        int rc = write_binary_level(img, &lv[l], b);
        if (rc) { free(nxt); free(b); return rc; }
        uint64_t o = 0;
        for (uint64_t i = 0; i < n; i++) if (!b[i]) nxt[o++] = cur[i];
        for (uint64_t i = 0; i < n; i++) if (b[i]) nxt[o++] = cur[i];
        memcpy(cur, nxt, n * sizeof(uint32_t));
    }
    free(nxt);
    free(b);
    return O_OK;
}

/* Balanced multiary tree of degree d = 2^D (Sec. 4.3): the full binary tree
 * over L_b = D*ceil(L/D) key bits (zero bits added at the top), keeping only
 * the levels beta*D.  Level beta holds, for the symbols in the order of that
 * binary level, the D key bits below the top beta*D bits. */
static int build_multi(uint8_t* img, olevel* lv, unsigned L, unsigned D,
                       uint32_t* cur, uint64_t n)
{
    unsigned M = (L + D - 1) / D, Lb = D * M;
    uint32_t d = 1u << D;
    uint32_t* nxt = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    uint8_t* g = (uint8_t*)malloc(n ? n : 1);
    if (!nxt || !g) { free(nxt); free(g); return O_ENOMEM; }
    for (unsigned be = 0; be < M; be++) {
        unsigned sh = Lb - D * (be + 1);
        for (uint64_t i = 0; i < n; i++) g[i] = (uint8_t)(((uint64_t)cur[i] >> sh) & (d - 1));
        write_multi_level(img, &lv[be], g, D);
        uint64_t s = 0;
        while (s < n) {
            uint64_t e = s + 1;
            if (be > 0) {
                uint64_t p = (uint64_t)cur[s] >> (Lb - D * be);
                while (e < n && ((uint64_t)cur[e] >> (Lb - D * be)) == p) e++;
            } else {
                e = n;
            }
            uint64_t o = s;
            for (uint32_t c = 0; c < d; c++)
                for (uint64_t i = s; i < e; i++) if (g[i] == c) nxt[o++] = cur[i];
            s = e;
        }
        memcpy(cur, nxt, n * sizeof(uint32_t));
    }
    free(nxt);
    free(g);
    return O_OK;
}

/* ---- shaped trees ------------------------------------------------------- */

typedef struct { uint32_t level; uint64_t prefix; } onode_key;

static int cmp_node_key(const void* a, const void* b)
{
    const onode_key* x = (const onode_key*)a;
    const onode_key* y = (const onode_key*)b;
    if (x->level != y->level) return x->level < y->level ? -1 : 1;
    if (x->prefix != y->prefix) return x->prefix < y->prefix ? -1 : 1;
    return 0;
}

/* index of (level, prefix) in the sorted node list, or -1 */
static int64_t find_node(const onode_key* nodes, uint64_t nn, uint32_t level, uint64_t prefix)
{
    uint64_t lo = 0, hi = nn;
    onode_key k = {level, prefix};
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        int c = cmp_node_key(&nodes[mid], &k);
        if (c == 0) return (int64_t)mid;
        if (c < 0) lo = mid + 1; else hi = mid;
    }
    return -1;
}

/* Arbitrary-shaped binary tree from codewords (Sec. 4.3): the codeword of a
 * symbol spells its root-to-leaf path, the i-th most significant bit being 0
 * when the path turns left.  The internal nodes at depth l are the proper
 * prefixes of length l of the codewords; level l holds, for every symbol
 * whose codeword is longer than l, bit l of its codeword, in the order of a
 * stable sort by the first l codeword bits (node order, left to right). */
/* The shaped tree of D-bit digits (D = 1: binary; Sec. 4.3, the shape
 * carried over to multiary trees): a codeword has lens[s] digits, digit l at
 * bits [D(lens-1-l), D(lens-l)) of codes[s].  Level l holds digit l of every
 * symbol whose codeword is longer than l, node by node in prefix order, in
 * input order inside a node. */
static uint64_t code_prefix(const uint64_t* codes, const uint32_t* lens, uint32_t s, unsigned l, unsigned D)
{
    return l ? (codes[s] >> (D * (lens[s] - l))) : 0;
}

static int build_shaped(uint8_t* img_or_null, olevel* lv, unsigned h, unsigned D,
                        const uint32_t* x, uint64_t n, uint32_t sigma,
                        const uint64_t* codes, const uint32_t* lens,
                        onode_key* nodes, uint64_t nnodes, uint8_t* node_rec)
{
    const uint64_t nb = node_bytes(D);
    const uint32_t d = 1u << D;
    /* cur: indices into x of the symbols on the current level */
    uint64_t* cur = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* nxt = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint8_t* b = (uint8_t*)malloc(n ? n : 1);
    if (!cur || !nxt || !b) { free(cur); free(nxt); free(b); return O_ENOMEM; }
    uint64_t m = n;
    for (uint64_t i = 0; i < n; i++) cur[i] = i;
    for (unsigned l = 0; l < h; l++) {
        if (m != lv[l].n) { free(cur); free(nxt); free(b); return O_EINVAL; }
        for (uint64_t k = 0; k < m; k++) {
            uint32_t s = x[cur[k]];
            b[k] = (uint8_t)((codes[s] >> (D * (lens[s] - 1 - l))) & (d - 1));
        }
        if (img_or_null) {
            if (D == 1) {
                int rc = write_binary_level(img_or_null, &lv[l], b);
                if (rc) { free(cur); free(nxt); free(b); return rc; }
            } else {
                write_multi_level(img_or_null, &lv[l], b, D);
            }
        }
        /* node records of depth l: start and count of every node segment */
        uint64_t s0 = 0;
        while (s0 < m) {
            uint32_t sy = x[cur[s0]];
            uint64_t p = code_prefix(codes, lens, sy, l, D);
            uint64_t e = s0 + 1;
            while (e < m) {
                uint32_t t = x[cur[e]];
                uint64_t q = code_prefix(codes, lens, t, l, D);
                if (q != p) break;
                e++;
            }
            int64_t id = find_node(nodes, nnodes, l, p);
            if (id < 0) { free(cur); free(nxt); free(b); return O_EINVAL; }
            put_u64(node_rec + (uint64_t)id * nb + 0, s0);
            put_u64(node_rec + (uint64_t)id * nb + 8, e - s0);
            s0 = e;
        }
        /* go down: stable partition inside each node, then drop the symbols
         * whose codeword ends at depth l+1 (they reached their leaf) */
        uint64_t o = 0;
        s0 = 0;
        while (s0 < m) {
            uint32_t sy = x[cur[s0]];
            uint64_t p = code_prefix(codes, lens, sy, l, D);
            uint64_t e = s0 + 1;
            while (e < m) {
                uint32_t t = x[cur[e]];
                uint64_t q = code_prefix(codes, lens, t, l, D);
                if (q != p) break;
                e++;
            }
            for (uint32_t digit = 0; digit < d; digit++)
                for (uint64_t k = s0; k < e; k++)
                    if (b[k] == digit && lens[x[cur[k]]] > l + 1) nxt[o++] = cur[k];
            s0 = e;
        }
        uint64_t* t = cur; cur = nxt; nxt = t;
        m = o;
    }
    (void)sigma;
    free(cur);
    free(nxt);
    free(b);
    return O_OK;
}

/* ---- canonical Huffman codes -------------------------------------------- */

typedef struct { uint64_t w; uint32_t sym; } oleaf;

static int cmp_leaf(const void* a, const void* b)
{
    const oleaf* x = (const oleaf*)a;
    const oleaf* y = (const oleaf*)b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

typedef struct { uint32_t len, sym; } olen;

static int cmp_len(const void* a, const void* b)
{
    const olen* x = (const olen*)a;
    const olen* y = (const olen*)b;
    if (x->len != y->len) return x->len < y->len ? -1 : 1;
    return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

/* Huffman code lengths by the two-queue method: leaves sorted by (count,
 * symbol) in one queue, merged nodes in creation order in the other; each
 * step merges the two lightest entries, taking the leaf on equal weight.
 * Symbols of count 0 get no code; a single coded symbol gets length 1.
 * Codes are then assigned canonically in (length, symbol) order. */
int oracle_huffman(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* lens)
{
    uint64_t k = 0;
    for (uint32_t s = 0; s < sigma; s++) { codes[s] = 0; lens[s] = 0; if (counts[s]) k++; }
    if (k == 0) return O_OK;
    if (k == 1) {
        for (uint32_t s = 0; s < sigma; s++) if (counts[s]) lens[s] = 1;
        return O_OK;
    }
    oleaf* leaves = (oleaf*)malloc(k * sizeof(oleaf));
    /* node ids: leaves 0..k-1, internal k..2k-2 */
    uint64_t* parent = (uint64_t*)malloc((2 * k - 1) * sizeof(uint64_t));
    uint64_t* iw = (uint64_t*)malloc((k - 1) * sizeof(uint64_t));
    uint32_t* depth = (uint32_t*)malloc((2 * k - 1) * sizeof(uint32_t));
    olen* order = (olen*)malloc(k * sizeof(olen));
    if (!leaves || !parent || !iw || !depth || !order) {
        free(leaves); free(parent); free(iw); free(depth); free(order);
        return O_ENOMEM;
    }
    uint64_t j = 0;
    for (uint32_t s = 0; s < sigma; s++)
        if (counts[s]) { leaves[j].w = counts[s]; leaves[j].sym = s; j++; }
    qsort(leaves, k, sizeof(oleaf), cmp_leaf);
    uint64_t lf = 0, inf = 0, ni = 0;   /* leaf front, internal front, internal count */
    for (uint64_t step = 0; step < k - 1; step++) {
        uint64_t pick[2];
        uint64_t wsum = 0;
        for (int t = 0; t < 2; t++) {
            int take_leaf = lf < k && (inf >= ni || leaves[lf].w <= iw[inf]);
            if (take_leaf) { pick[t] = lf; wsum += leaves[lf].w; lf++; }
            else { pick[t] = k + inf; wsum += iw[inf]; inf++; }
        }
        iw[ni] = wsum;
        parent[pick[0]] = k + ni;
        parent[pick[1]] = k + ni;
        ni++;
    }
    /* the root is the last internal node; parents are created after children */
    depth[2 * k - 2] = 0;
    for (int64_t v = (int64_t)(2 * k - 3); v >= 0; v--) depth[v] = depth[parent[v]] + 1;
    for (uint64_t t = 0; t < k; t++) {
        lens[leaves[t].sym] = depth[t];
        order[t].len = depth[t];
        order[t].sym = leaves[t].sym;
    }
    qsort(order, k, sizeof(olen), cmp_len);
    uint64_t code = 0;
    for (uint64_t t = 0; t < k; t++) {
        if (t > 0) code = (code + 1) << (order[t].len - order[t - 1].len);
        codes[order[t].sym] = code;
    }
    free(leaves); free(parent); free(iw); free(depth); free(order);
    return O_OK;
}

/* ---- entry point -------------------------------------------------------- */

void oracle_free(void* p) { free(p); }

/* Build the structure of the given kind over S and return its canonical image
 * (malloc'ed, free with oracle_free).  codes/lens are used by the shaped kind
 * only (arrays of sigma entries; lens[s] == 0 means s has no codeword). */
int oracle_build(int kind, const void* S, int sym_bytes, uint64_t n, uint32_t sigma,
                 int arity_log2, const uint64_t* codes, const uint32_t* lens,
                 uint8_t** image, uint64_t* image_bytes)
{
    *image = NULL;
    *image_bytes = 0;
    if (sigma == 0) return O_EINVAL;
    if (kind < O_KIND_WT || kind > O_KIND_MULTI) return O_EINVAL;
    if (kind == O_KIND_SHAPED && arity_log2 == 0) arity_log2 = 1;   /* binary */
    if ((kind == O_KIND_MULTI || kind == O_KIND_SHAPED) && (arity_log2 < 1 || arity_log2 > 4)) return O_EINVAL;
    if (kind != O_KIND_MULTI && kind != O_KIND_SHAPED) arity_log2 = 1;
    if (kind == O_KIND_SHAPED && (!codes || !lens)) return O_EINVAL;

    uint32_t* x = NULL;
    int rc = read_symbols(S, sym_bytes, n, sigma, &x);
    if (rc) return rc;

    unsigned L = key_bits_of(sigma);
    unsigned D = (unsigned)arity_log2;
    unsigned nlev = 0, key_bits = 0;
    uint64_t nnodes = 0, ncoded = 0;
    onode_key* nodes = NULL;
    olevel lv[64];
    memset(lv, 0, sizeof(lv));

    if (kind == O_KIND_WT || kind == O_KIND_WM) {
        nlev = L;
        key_bits = L;
        for (unsigned l = 0; l < nlev; l++) lv[l].n = n;
    } else if (kind == O_KIND_MULTI) {
        nlev = (L + D - 1) / D;
        key_bits = D * nlev;
        for (unsigned l = 0; l < nlev; l++) lv[l].n = n;
    } else {
        /* code lengths count D-bit digits; at most 32 bits per codeword */
        unsigned h = 0;
        for (uint32_t s = 0; s < sigma; s++) {
            if ((uint64_t)lens[s] * D > O_MAX_CODE_LEN) { free(x); return O_EUNSUP; }
            if (lens[s]) { ncoded++; if (lens[s] > h) h = lens[s]; }
        }
        for (uint64_t i = 0; i < n; i++)
            if (lens[x[i]] == 0) { free(x); return O_ERANGE; }
        if (h == 0) { free(x); return O_EINVAL; }
        nlev = h;
        key_bits = h * D;
        for (uint64_t i = 0; i < n; i++)
            for (unsigned l = 0; l < lens[x[i]]; l++) lv[l].n++;
        /* internal nodes: proper prefixes of the codewords */
        uint64_t cap = 0;
        for (uint32_t s = 0; s < sigma; s++) cap += lens[s];
        nodes = (onode_key*)malloc((cap ? cap : 1) * sizeof(onode_key));
        if (!nodes) { free(x); return O_ENOMEM; }
        for (uint32_t s = 0; s < sigma; s++)
            for (unsigned l = 0; l < lens[s]; l++) {
                nodes[nnodes].level = l;
                nodes[nnodes].prefix = code_prefix(codes, lens, s, l, D);
                nnodes++;
            }
        qsort(nodes, nnodes, sizeof(onode_key), cmp_node_key);
        uint64_t u = 0;
        for (uint64_t t = 0; t < nnodes; t++)
            if (u == 0 || cmp_node_key(&nodes[u - 1], &nodes[t]) != 0) nodes[u++] = nodes[t];
        nnodes = u;
    }

    uint64_t nodes_off = 0, codes_off = 0;
    const int multi_levels = kind == O_KIND_MULTI || (kind == O_KIND_SHAPED && D >= 2);
    uint64_t total = lay_out(lv, nlev, multi_levels, D, nnodes, sigma,
                             kind == O_KIND_SHAPED, &nodes_off, &codes_off);
    uint8_t* img = (uint8_t*)calloc(1, total);
    if (!img) { free(x); free(nodes); return O_ENOMEM; }

    if (kind == O_KIND_WT) rc = build_wt(img, lv, L, x, n);
    else if (kind == O_KIND_WM) rc = build_wm(img, lv, L, x, n);
    else if (kind == O_KIND_MULTI) rc = build_multi(img, lv, L, D, x, n);
    else {
        uint8_t* rec = img + nodes_off;
        const uint64_t nb = node_bytes(D);
        const uint32_t d = 1u << D;
        /* every node starts empty at the position its symbols would take */
        rc = build_shaped(img, lv, nlev, D, x, n, sigma, codes, lens, nodes, nnodes, rec);
        if (rc == O_OK) {
            /* empty nodes (codewords of absent symbols): start = number of
             * level-l symbols whose l-digit prefix is smaller */
            for (uint64_t t = 0; t < nnodes; t++) {
                uint64_t cnt;
                memcpy(&cnt, rec + t * nb + 8, 8);
                if (cnt) continue;
                uint64_t before = 0;
                for (uint64_t i = 0; i < n; i++) {
                    uint32_t s = x[i];
                    unsigned l = nodes[t].level;
                    if (lens[s] > l && code_prefix(codes, lens, s, l, D) < nodes[t].prefix) before++;
                }
                put_u64(rec + t * nb + 0, before);
            }
            /* children: an internal node, a leaf (a symbol whose codeword is
             * this prefix), or none */
            for (uint64_t t = 0; t < nnodes; t++) {
                uint8_t* e = rec + t * nb;
                for (uint32_t c = 0; c < d; c++) {
                    uint32_t l1 = nodes[t].level + 1;
                    uint64_t q = nodes[t].prefix * d + (uint64_t)c;
                    uint32_t child = O_NO_CHILD;
                    int64_t id = find_node(nodes, nnodes, l1, q);
                    if (id >= 0) {
                        child = (uint32_t)id;
                    } else {
                        for (uint32_t s = 0; s < sigma; s++)
                            if (lens[s] == l1 && codes[s] == q) { child = O_LEAF_FLAG | s; break; }
                    }
                    put_u32(e + (D == 1 ? 16 : 24) + 4 * c, child);
                }
                put_u32(e + (D == 1 ? 24 : 16), nodes[t].level);
                put_u32(e + (D == 1 ? 28 : 20), (uint32_t)nodes[t].prefix);
            }
            for (uint32_t s = 0; s < sigma; s++) {
                put_u64(img + codes_off + (uint64_t)s * O_CODE_BYTES, lens[s] ? codes[s] : 0);
                put_u32(img + codes_off + (uint64_t)s * O_CODE_BYTES + 8, lens[s]);
            }
        }
    }
    if (rc) { free(img); free(x); free(nodes); return rc; }
    write_header(img, kind, D, n, sigma, nlev, key_bits, total, nodes_off, nnodes,
                 codes_off, ncoded, lv);
    free(x);
    free(nodes);
    *image = img;
    *image_bytes = total;
    return O_OK;
}
