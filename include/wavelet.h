/*
 * wavelet.h -- C-ABI of the MI355X wavelet tree / wavelet matrix builder.
 *
 * Builds, on one AMD Instinct MI355X (gfx950), the structures of Shun,
 * "Improved Parallel Construction of Wavelet Trees and Rank/Select
 * Structures", over an integer sequence S of n symbols drawn from the
 * alphabet [0, sigma-1] (Sec. 2, problem statement):
 *
 *   kind WT_KIND_WT        balanced binary wavelet tree, levelwise and
 *                          pointerless (Sec. 2, recursive definition)
 *   kind WT_KIND_WM        wavelet matrix (Sec. 4.3, "Wavelet matrix")
 *   kind WT_KIND_SHAPED    binary tree shaped by given codewords, e.g.
 *                          Huffman-shaped (Sec. 4.3, "Arbitrarily-shaped")
 *   kind WT_KIND_MULTIARY  balanced multiary tree of degree d = 2^D,
 *                          D in 1..4 (Sec. 4.3, "Multiary wavelet trees")
 *
 * Every binary level carries a rank-of-0 directory (Sec. 5.1, "Rank": 512-bit
 * ranges, 64-bit sub-ranges) and sampled select on ones and zeros (Sec. 5.1,
 * "Select": the two sampling levels of Clark's structure, every 4096th and
 * every 512th one/zero, and Clark's rule for long ranges: the 512 answers of
 * a stretch between two sub-samples spanning 2^20 bits or more are stored,
 * any other stretch is searched in the rank ranges); multiary levels carry
 * per-digit
 * rank counters (Sec. 5.2, "Rank").
 *
 * Output: one flat, position-independent byte image per structure (layout
 * below).  The image only holds offsets, so it can be copied, saved and
 * reloaded as is.
 *
 * Conventions shared by every call:
 *   - "dev" pointers are device memory (hipMalloc'ed or torch CUDA tensors);
 *     "host" pointers are ordinary host memory.  All buffers are owned by the
 *     caller; the library never allocates device memory on the build path.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Build and query calls are asynchronous on `stream` unless stated.
 *   - Return value: WT_OK or a negative WT_E* code.  Argument errors are
 *     reported before anything is launched.  A symbol >= sigma is found on
 *     the device: the build then marks the image header and wt_check()
 *     returns WT_ERANGE (the rest of the image is unspecified); a shaped
 *     tree whose sequence has other counts than shape->counts is marked the
 *     same way and wt_check() returns WT_EINVAL.
 *   - Builds do not wait on the host (except balanced and multiary trees
 *     over more than 20 key bits, which read the symbol counts back, and the
 *     level-by-level tree path, below), so a caller may capture any other
 *     build into a HIP graph.
 *   - Limits: n < 2^32, sigma >= 1, sym_bytes in {1, 2, 4}, at most 32
 *     levels, codeword length <= 32.
 */
#ifndef WAVELET_H
#define WAVELET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define WT_OK       0
#define WT_EINVAL  (-1)   /* bad n / sigma / width / shape / pointer       */
#define WT_ERANGE  (-2)   /* a symbol >= sigma (or without codeword) seen  */
#define WT_ENOSPC  (-3)   /* output or workspace buffer too small          */
#define WT_EHIP    (-4)   /* a HIP runtime call failed                     */
#define WT_EUNSUP  (-5)   /* outside the supported limits                  */

/* ---- kinds -------------------------------------------------------------- */
#define WT_KIND_WT        1
#define WT_KIND_WM        2
#define WT_KIND_SHAPED    3
#define WT_KIND_MULTIARY  4

/* ---- image layout (little endian) ----------------------------------------
 * Header, 256 bytes at offset 0:
 *   u32 magic 0x54564157 ("WAVT"), u32 version 3, u32 kind, u32 arity_log2,
 *   u64 n, u32 sigma, u32 nlevels, u32 key_bits, u32 status (0 ok; bit 0:
 *   a symbol >= sigma was seen; bit 1: the symbol counts differ from those
 *   the shape gave), u64 image_bytes, u64 levels_off (= 256),
 *   u64 nodes_off, u64 nnodes, u64 codes_off, u64 ncoded; rest zero.
 * Level descriptors, 64 bytes each, at levels_off + 64*l:
 *   u64 n_l, u64 zeros, u64 ones, u64 bits_off, u64 rank_off, u64 sel0_off,
 *   u64 sel1_off, u64 nsel.   (multiary: zeros = ones = sel1_off = 0;
 *   sel0_off = the per-digit select samples, nsel entries per digit value)
 * Arrays, each starting on a 256-byte boundary, level after level:
 *   binary level  bits: ceil(n_l/64) u64 words, bit i at bit (i%64) of word
 *                 i/64 (LSB first), padding bits 0;
 *                 rank: ceil(n_l/512)+1 pairs {u64 sb0, u64 blk}: sb0[k] =
 *                 zeros in [0, min(512k, n_l)); blk[k] = sum over j = 1..7 of
 *                 (zeros in [512k, min(512k+64j, n_l))) << 9(j-1), 0 when
 *                 512k >= n_l;
 *                 sel0 / sel1: nsel = ceil(n_l/4096)+1 u64: position of the
 *                 zero / one whose 0-based ordinal is 4096k, then n_l;
 *                 sub (at sel1_off + 8*nsel rounded up to 256 bytes, not in
 *                 the descriptor): nsub = ceil(n_l/512)+2 u32: entry j = the
 *                 position of the one of ordinal 512j, entry nsub-1-j = that
 *                 of the zero of ordinal 512j, every other entry n_l (at
 *                 least one such entry separates the two);
 *                 pool (at the end of sub rounded up to 256 bytes): 2 x
 *                 nslot slots of 512 u32, nslot = floor(n_l / 2^20), the
 *                 ones' slots then the zeros'.  When the one of ordinal 512j
 *                 sits at p and the one of ordinal 512(j+1) (n_l if none) at
 *                 least 2^20 bits later, slot floor(p / 2^20) holds the
 *                 positions of the ones of ordinals 512j, 512j+1, ... (no
 *                 two such stretches share a slot); the same for zeros;
 *                 every other entry n_l.
 *   multiary level (D-bit digits, P = floor(64/D) per word, digit t at bits
 *                 [tD, tD+D) of word t/P): ceil(n_l/P) words; then counters:
 *                 (ceil(n_l/64P)+1) x d u64 = count of each digit before
 *                 every 64-word range (last entry = totals), followed by
 *                 ceil(n_l/8P) x d u16 = count of each digit from the start
 *                 of its range to the start of every 8-word sub-range;
 *                 then the generalized select samples (Sec. 5.2, "Select"):
 *                 for every digit value c (c-major) nsel = ceil(n_l/4096)+1
 *                 u64: position of the c of 0-based ordinal 4096k, then n_l.
 *   shaped trees  node table (one record per internal node, ordered by
 *                 (level, prefix)): binary codes, 32 B: u64 start in its
 *                 level, u64 count, u32 child[2] (node index, or
 *                 0x80000000|symbol for a leaf, 0xFFFFFFFF if absent),
 *                 u32 level, u32 prefix; codes of D-bit digits (D >= 2),
 *                 24 + 4*2^D B: u64 start, u64 count, u32 level, u32 prefix,
 *                 u32 child[2^D]; then the code table (16 B per symbol): u64
 *                 codeword, u32 length in digits (0 = none), u32 0.  A shaped
 *                 tree over D-bit digits has multiary levels (as above, with
 *                 the level sizes of its codewords) and arity_log2 = D in
 *                 its header.
 * Bytes outside every array are zero.  Balanced trees (Sec. 2): level l is
 * the concatenation of the node bitstrings of depth l, left to right, every
 * level has n bits.  Wavelet matrix: level l is bit l from the top of the
 * symbols in the order of level l, zeros counted in `zeros` (Sec. 4.3).
 * ------------------------------------------------------------------------ */

typedef struct wt_shape {
    uint32_t arity_log2;       /* multiary: D in 1..4; shaped: 0 or 1 for
                                  binary codewords, 2..4 for codewords of
                                  D-bit digits (a shaped multiary tree, the
                                  shape carried over to multiary trees,
                                  Sec. 4.3); WT/WM: 0 or 1                  */
    uint32_t reserved;
    const uint64_t* codes;     /* shaped: host [sigma], codeword value, its
                                  i-th most significant digit (of code_len
                                  digits of D bits; D = 1 binary) is the
                                  child taken at depth i (binary: 0 = left)
                                  (Sec. 4.3, "Arbitrarily-shaped")          */
    const uint32_t* code_len;  /* shaped: host [sigma], length in digits, 0 =
                                  no codeword; code_len * D <= 32           */
    const uint64_t* counts;    /* shaped: host [sigma], occurrences of every
                                  symbol in S (fixes the level sizes)       */
} wt_shape;

typedef struct wt_tuning {
    uint32_t tau;      /* key bits per partition pass, 1..8 (0 = automatic) */
    uint32_t tile;     /* tiles of 8192 keys per chunk (0 = automatic);
                          ignored when `blocks` is set                      */
    uint32_t blocks;   /* chunks (workgroups) per pass (0 = automatic: one
                          per tile, at most the resident pass workgroups:
                          1024 = 4 per CU when the first pass's keys fit 16
                          bits, else 768 = 3 per CU; a batch without `tile`
                          sizes its chunks by the whole batch: up to 16
                          tiles, while every resident pass workgroup still
                          gets about 4 chunks)                              */
    uint32_t flags;    /* WT_FLAG_*                                         */
} wt_tuning;

/* force the level-by-level path (one level per pass) for any kind */
#define WT_FLAG_LEVELWISE 1u
/* time every kernel of the build with HIP events (read by wt_profile_read) */
#define WT_FLAG_PROFILE   2u

typedef struct wt_plan_info {
    uint32_t kind, nlevels, key_bits, arity_log2;
    uint64_t n;
    uint32_t sigma, tau;
    uint64_t out_bytes;        /* size of the canonical image              */
    uint64_t workspace_bytes;  /* device scratch the build needs           */
    uint64_t level_n[32];      /* bits / digits per level                  */
    /* shaped trees built from two matrices: the levels above split_bits
     * (key bits; for codewords of D-bit digits the digit levels above
     * split_bits / D) from a matrix over the top split_bits bits of every
     * padded codeword, the deeper levels from a matrix over the split_long
     * symbols with longer codes (chosen when those are at most 1/8 of S);
     * 0, 0: one matrix or none                                            */
    uint32_t split_bits, reserved0;
    uint64_t split_long;
} wt_plan_info;

/* Size a build (Sec. 2 problem statement; host only, no device work).
 * shape: NULL for WT/WM; codes+code_len+counts for SHAPED (the codewords
 * must be prefix-free, else WT_EINVAL; a code over D-bit digits when
 * arity_log2 >= 2, built level by level); arity for MULTIARY.  tune may be
 * NULL.  Fills *info. */
int wt_plan(int kind, uint64_t n, uint32_t sigma, uint32_t sym_bytes,
            const wt_shape* shape, const wt_tuning* tune, wt_plan_info* info);

/* Build a balanced binary wavelet tree (Sec. 2), or, when shape->codes is
 * set, the tree shaped by those codewords (Sec. 4.3, Thm. 4.4).
 * S: dev, n symbols of sym_bytes each.  out: dev, out_bytes >= plan
 * out_bytes, receives the image.  ws: dev scratch of ws_bytes >= plan
 * workspace_bytes.  S, out and ws must be 16-byte aligned (device
 * allocations are), else WT_EINVAL before any device work.  Asynchronous on
 * `stream`: a balanced tree derives the place of every run from the symbol
 * counts on the device (key bits <= 20; a wider alphabet reads the counts
 * back and waits, as does the level-by-level path); a shaped tree places its
 * runs from shape->counts on the host before launching, uploads its tables
 * from pinned host buffers that return to the library's pool once `stream`
 * has passed them (kept for good when `stream` is being captured), and the
 * device checks the counts (wt_check: WT_EINVAL if they differ).  A shaped
 * tree split into two matrices builds the smaller one on a second stream
 * the library keeps per device, forked from and joined back into `stream`
 * with events; split builds of different callers share that stream, so one
 * of them must not be captured into a graph while another is being built. */
int wt_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes,
             const wt_shape* shape, const wt_tuning* tune,
             void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream);

/* Build a wavelet matrix (Sec. 4.3, Thm. 4.6).  Same arguments as wt_build;
 * shape must be NULL. Fully asynchronous. */
int wm_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes,
             const wt_shape* shape, const wt_tuning* tune,
             void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream);

/* Build a balanced multiary wavelet tree of degree 2^shape->arity_log2
 * (Sec. 4.3, Thm. 4.5) with per-digit rank counters (Sec. 5.2).  Same
 * arguments as wt_build; asynchronous in the same way for D = 1, 2, 4
 * (8-ary trees take the level-by-level path, which waits for the counts
 * and returns WT_ERANGE directly). */
int multiary_build(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes,
                   const wt_shape* shape, const wt_tuning* tune,
                   void* out, size_t out_bytes, void* ws, size_t ws_bytes, void* stream);

/* Wavelet matrix build for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same build and image as wm_build, with the workspace taken
 * from a library-owned device array of WT_NOALLOC_SCRATCH_BYTES per GPU
 * (placed when the library is loaded on that GPU and held until the process
 * ends) instead of a caller buffer.  S and out as for wm_build; no tuning
 * flags beyond tau / blocks / WT_FLAG_LEVELWISE (WT_FLAG_PROFILE is ignored).
 * Returns WT_ENOSPC, before any device work, when the build needs more
 * workspace than the array holds (about n <= 2^22 symbols of 32 bits; the
 * bound is the plan's workspace_bytes).  Calls no allocating routine.  Every
 * call on one GPU uses that GPU's one array, so calls that overlap on one GPU
 * (on different streams, or from different threads) race and must be
 * serialized by the caller; each call writes every workspace byte it reads
 * before reading it. */
#define WT_NOALLOC_SCRATCH_BYTES (64u << 20)
int wm_build_noalloc(const void* S, uint64_t n, uint32_t sigma, uint32_t sym_bytes,
                     const wt_tuning* tune, void* out, size_t out_bytes, void* stream);

/* Synchronize `stream` and read the status word of a built image (dev).
 * Returns WT_OK; WT_ERANGE if a symbol >= sigma was seen; WT_EINVAL if a
 * shaped tree's symbol counts differ from shape->counts. */
int wt_check(const void* image, void* stream);

/* Batched queries on a built image (dev), m queries, all arrays dev.
 * access (Sec. 2): res[q] = S[pos[q]], UINT32_MAX if pos[q] >= n.
 * rank   (Sec. 2): res[q] = occurrences of c[q] in S[0..i[q]] (inclusive);
 *                  0 if c[q] >= sigma or has no codeword; UINT64_MAX if
 *                  i[q] >= n.
 * select (Sec. 2): res[q] = position of the k[q]-th occurrence of c[q]
 *                  (k 1-based); UINT64_MAX if k = 0, k > count or c invalid.
 * One launch per call: m > 2^39 - 256 queries returns WT_EUNSUP before any
 * device work. */
int wt_access(const void* image, const uint64_t* pos, uint32_t* res, uint64_t m, void* stream);
int wt_rank(const void* image, const uint32_t* c, const uint64_t* i, uint64_t* res,
            uint64_t m, void* stream);
int wt_select(const void* image, const uint32_t* c, const uint64_t* k, uint64_t* res,
              uint64_t m, void* stream);

/* Occurrences of every symbol of S (dev) into counts (dev, sigma u64), e.g.
 * to build Huffman codewords; symbols >= sigma are not counted. */
int wt_symbol_counts(const void* S, uint64_t n, uint32_t sym_bytes, uint32_t sigma,
                     uint64_t* counts, void* stream);

/* Canonical Huffman codewords from counts (all host arrays of sigma).
 * Two-queue merge with leaves ordered by (count, symbol), the leaf taken on
 * equal weight; codes assigned in (length, symbol) order; a single coded
 * symbol gets length 1; count 0 gets length 0.  WT_EUNSUP if a length
 * exceeds 32. */
int wt_huffman_codes(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* code_len);

/* The same codewords computed on the device (the paper notes Huffman
 * codewords can be generated in parallel, Sec. 4.3), from device counts,
 * e.g. those of wt_symbol_counts: counts, codes, code_len (sigma entries
 * each) and status (one entry) are dev arrays; asynchronous on `stream`, one
 * workgroup, no workspace.  *status becomes WT_OK, or WT_EUNSUP when a length
 * exceeds 32 (codes and lengths then 0).  Returns WT_EUNSUP for sigma above
 * WT_HUFFMAN_DEV_MAX_SIGMA (use wt_huffman_codes), WT_EINVAL for sigma 0 or
 * a null pointer. */
#define WT_HUFFMAN_DEV_MAX_SIGMA 4096u
int wt_huffman_codes_dev(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* code_len,
                         int32_t* status, void* stream);

/* One sequence of a batched build.  S, out: dev pointers, 16-byte aligned
 * (as is the batch workspace; else WT_EINVAL).  tau: key bits
 * per pass for this sequence (0 = the batch tuning, else automatic); the
 * image does not depend on it. */
typedef struct wt_seq_desc {
    const void* S;
    uint64_t n;
    uint32_t sigma;
    uint32_t sym_bytes;
    void* out;
    uint64_t out_bytes;
    uint32_t tau;
    uint32_t reserved;
} wt_seq_desc;

/* Size of the workspace a batched build of `count` sequences needs. */
int wt_batch_plan(int kind, const wt_seq_desc* seqs, uint32_t count, const wt_tuning* tune,
                  uint64_t* workspace_bytes);

/* Build wavelet matrices (kind WT_KIND_WM) of many sequences with a few
 * persistent launches; each image equals the one wm_build writes for that
 * sequence alone.  seqs: host array of count descriptors (read during the
 * call only).  Asynchronous on `stream`: every descriptor of the batch is
 * written into a pinned host buffer before the first launch and one kernel
 * copies it into ws; the buffer returns to the library's pool once `stream`
 * has passed that copy (kept for good when `stream` is being captured).
 * Launches per batch: 2 + 4 per group + 3, a group being the sequences of
 * one round of passes whose keys fit 16 bits, or those whose keys do not
 * (a round of passes holds every sequence with levels left to build).
 * tune->tile: tiles per chunk for every sequence of the batch. */
int wt_batch_build(int kind, const wt_seq_desc* seqs, uint32_t count,
                   void* ws, size_t ws_bytes, const wt_tuning* tune, void* stream);

/* Bytes of a built image (reads the header; dev image, synchronizes). */
int wt_image_bytes(const void* image, uint64_t* bytes, void* stream);

/* Per-kernel timing of builds run with WT_FLAG_PROFILE: synchronizes the
 * recorded events and returns, per kernel name, the number of launches and
 * their summed duration (ms) since the last call; resets the totals.
 * out: host array of cap entries; *count = number of names (may exceed cap). */
typedef struct wt_profile_entry {
    char name[48];
    uint64_t launches;
    double ms;
} wt_profile_entry;
int wt_profile_read(wt_profile_entry* out, uint32_t cap, uint32_t* count);

/* Human-readable text of a status code. */
const char* wt_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* WAVELET_H */
