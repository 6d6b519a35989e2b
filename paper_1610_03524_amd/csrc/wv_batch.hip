// wv_batch.hip -- wavelet matrices of many sequences with a few persistent
// launches.
//
// Every sequence is built with the passes of wm_build and into the image
// wm_build writes (chunks are sized by the whole batch), but each step runs
// for all sequences in one launch: the chunk histograms of every sequence, their prefix over the
// chunks, every chunk's run offsets, then a persistent pass
// kernel whose workgroups pull chunks of any sequence from a device-side
// queue (largest sequences first), and finally the directories of every
// level of every sequence.  Sequences with more levels take more rounds of
// passes; a round only holds the sequences that still have levels to build.
// The host writes the descriptors of every phase into one pinned buffer
// before the first launch; one kernel copies them to the workspace, and the
// call returns once everything is queued (stream-ordered, so a batch can be
// captured in a graph).  Launches: the copy, the headers (which also clear
// the histogram area and the work queues), four per group of a round
// (histograms, their prefix, run offsets, the persistent pass, which clears
// the histogram area again for the next group) and three for the
// directories.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "wv_wm_core.h"
#include "wv_wm_passes.h"

namespace {

struct SeqRound {
    PassArgs pa;            // the pass of this round (G0 points to the sequence's table)
    uint32_t* H;            // [2^tau][K] digit counts of the chunks
    uint32_t* tot;          // [2^tau] digit totals
    uint32_t* status;       // image status word (first round) or null
    uint32_t in_bytes, out_bytes, sigma, chunk0;   // chunk0: first global chunk index
    uint32_t col0;          // first global (sequence, digit) column
};

struct SpanDesc {
    uint8_t* image;
    uint64_t n, bits_off, rank_off, sel0_off, sel1_off, nsel, sub_off, nsub;
    uint32_t* cnt;          // ones per directory chunk
    uint64_t* pre;          // exclusive prefix of cnt
    uint32_t level, chunk0; // level index, first directory workgroup of the span
};

constexpr uint32_t SDW = 512;   // words per directory chunk
constexpr uint32_t SDG = 8;     // directory chunks per workgroup (one descriptor search each)

// grid-stride clear of count words (every workgroup of the launch takes part)
__device__ inline void grid_zero(uint32_t* p, uint64_t count)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// global item -> owner, over an exclusive prefix array of `count` owners
__device__ inline uint32_t owner_of(const uint32_t* first, uint32_t count, uint32_t item)
{
    uint32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(HT)
b_hist_k(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ chunk0, uint32_t nseq)
{
    __shared__ uint32_t h[HWORDS];
    const uint32_t item = blockIdx.x / HSPLIT, part = blockIdx.x % HSPLIT;
    const uint32_t s = owner_of(chunk0, nseq, item);
    const SeqRound& q = seqs[s];
    const uint32_t b = item - q.chunk0;
    const PassArgs& a = q.pa;
    if (q.in_bytes == 1)
        wm_hist_part<uint8_t>(a.in, a.n, a.C, a.K, a.R, a.tau, a.keymask, q.H, q.status, q.sigma, b, part, h);
    else if (q.in_bytes == 2)
        wm_hist_part<uint16_t>(a.in, a.n, a.C, a.K, a.R, a.tau, a.keymask, q.H, q.status, q.sigma, b, part, h);
    else
        wm_hist_part<uint32_t>(a.in, a.n, a.C, a.K, a.R, a.tau, a.keymask, q.H, q.status, q.sigma, b, part, h);
}

// exclusive prefix over the chunks of every (sequence, digit) column of H,
// one wave per column; the column sums go to the sequence's totals
__global__ void __launch_bounds__(HT)
b_scan_k(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ col0, uint32_t nseq, uint32_t ncols)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t item = blockIdx.x * (HT / 64) + (threadIdx.x >> 6);
    if (item >= ncols) return;   // whole waves; no barriers below
    const uint32_t s = owner_of(col0, nseq, item);
    const SeqRound& q = seqs[s];
    const uint32_t d = item - col0[s], K = q.pa.K;
    uint32_t* h = q.H + (uint64_t)d * K;
    uint32_t run = 0;
    for (uint32_t base = 0; base < K; base += 64) {
        const uint32_t i = base + lane;
        const uint32_t v = i < K ? h[i] : 0u;
        uint32_t t;
        const uint32_t ex = wave_excl_scan(v, &t);
        if (i < K) h[i] = run + ex;
        run += t;
    }
    if (lane == 0) q.tot[d] = run;
}

// one workgroup per chunk of any sequence: the chunk's run offsets (and
// zeroed boundary words)
__global__ void __launch_bounds__(HT)
b_offsets_k(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ chunk0, uint32_t nseq)
{
    __shared__ OffShared sh;
    const uint32_t s = owner_of(chunk0, nseq, blockIdx.x);
    const SeqRound& q = seqs[s];
    const PassArgs& a = q.pa;
    const uint32_t b = blockIdx.x - q.chunk0, tau = a.tau;
    if (threadIdx.x < (1u << tau)) {
        sh.cj[gidx(tau, threadIdx.x)] = q.H[(uint64_t)threadIdx.x * a.K + b];
        sh.tj[gidx(tau, threadIdx.x)] = q.tot[threadIdx.x];
    }
    wm_chunk_offsets(sh, b, tau, a.n, (uint32_t*)a.G0, a.words);
}

// persistent pass: workgroups take chunks from the queue until it is empty,
// then clear the histogram area for the next group (its histograms were read
// by the offsets launch before this one)
template <typename KT_>
__device__ void b_pass_body(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ chunk0, uint32_t nseq,
                            uint32_t nchunks, uint32_t* __restrict__ queue, uint32_t* __restrict__ zero,
                            uint64_t nzero, PassShared<KT_>& sh, uint32_t& item_s)
{
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(queue, 1u);
        __syncthreads();
        // uniform across the workgroup: the descriptor loads below are scalar
        const uint32_t item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item_s);
        __syncthreads();
        if (item >= nchunks) break;
        const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)owner_of(chunk0, nseq, item));
        const SeqRound& q = seqs[s];
        const uint32_t b = item - q.chunk0;
        // any input width (the first pass reads S as stored) and payload
        // width: both are read at run time, so the kernel holds one copy of
        // the pass
        wm_pass_chunk<KT_>(q.pa, b, sh);
        __syncthreads();
    }
    grid_zero(zero, nzero);
}

// 16-bit keys in LDS: four workgroups per CU; 32-bit keys: three (LDS-bound)
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8)))
b_pass16_k(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ chunk0, uint32_t nseq,
           uint32_t nchunks, uint32_t* __restrict__ queue, uint32_t* __restrict__ zero, uint64_t nzero)
{
    __shared__ PassShared<uint16_t> sh;
    __shared__ uint32_t item_s;
    b_pass_body<uint16_t>(seqs, chunk0, nseq, nchunks, queue, zero, nzero, sh, item_s);
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 6)))
b_pass32_k(const SeqRound* __restrict__ seqs, const uint32_t* __restrict__ chunk0, uint32_t nseq,
           uint32_t nchunks, uint32_t* __restrict__ queue, uint32_t* __restrict__ zero, uint64_t nzero)
{
    __shared__ PassShared<uint32_t> sh;
    __shared__ uint32_t item_s;
    b_pass_body<uint32_t>(seqs, chunk0, nseq, nchunks, queue, zero, nzero, sh, item_s);
}


// ---- directories of every (sequence, level) ------------------------------------

__global__ void __launch_bounds__(256)
b_dir_count_k(const SpanDesc* __restrict__ spans, const uint32_t* __restrict__ chunk0, uint32_t nspan)
{
    __shared__ uint32_t part[SDG][4];
    const uint32_t s = owner_of(chunk0, nspan, blockIdx.x);
    const SpanDesc& d = spans[s];
    const uint64_t nw = wv_cdiv(d.n, 64), nch = wv_cdiv(nw, SDW);
    const uint64_t c0 = (uint64_t)(blockIdx.x - d.chunk0) * SDG;
    const uint64_t* words = (const uint64_t*)(d.image + d.bits_off);
    // the SDG chunks' words in flight together (index clamped, masked after)
    uint64_t x[SDG][2];
#pragma unroll
    for (uint32_t g = 0; g < SDG; g++) {
        const uint64_t w0 = (c0 + g) * SDW + 2 * threadIdx.x;
        x[g][0] = words[min(w0, nw - 1)];
        x[g][1] = words[min(w0 + 1, nw - 1)];
    }
#pragma unroll
    for (uint32_t g = 0; g < SDG; g++) {
        const uint64_t w0 = (c0 + g) * SDW + 2 * threadIdx.x;
        uint32_t o = (w0 < nw ? (uint32_t)__popcll(x[g][0]) : 0u) + (w0 + 1 < nw ? (uint32_t)__popcll(x[g][1]) : 0u);
        o = wv_wave_incl_scan(o);   // lane 63 holds the wave's sum
        if ((threadIdx.x & 63) == 63) part[g][threadIdx.x >> 6] = o;
    }
    __syncthreads();
    if (threadIdx.x < SDG && c0 + threadIdx.x < nch)
        d.cnt[c0 + threadIdx.x] = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] + part[threadIdx.x][3];
}

__global__ void __launch_bounds__(256)
b_dir_scan_k(const SpanDesc* __restrict__ spans)
{
    __shared__ uint32_t ws[4];
    __shared__ uint64_t total_s;
    const SpanDesc& d = spans[blockIdx.x];
    const uint64_t nch = wv_cdiv(wv_cdiv(d.n, 64), SDW);
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t run = 0;
    for (uint64_t base = 0; base < nch; base += 256) {
        const uint64_t i = base + threadIdx.x;
        const uint32_t v = i < nch ? d.cnt[i] : 0u;
        uint32_t wt;
        const uint32_t ex = wave_excl_scan(v, &wt);
        if (lane == 0) ws[wave] = wt;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (uint32_t k = 0; k < 4; k++) {
            if (k < wave) off += ws[k];
            tot += ws[k];
        }
        if (i < nch) d.pre[i] = run + off + ex;
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) total_s = run;
    __syncthreads();
    const uint64_t ones = total_s, zeros = d.n - ones, ns = wv_cdiv(d.n, WV_SB_BITS);
    uint64_t* dir = (uint64_t*)(d.image + d.rank_off);
    uint64_t* sel0 = (uint64_t*)(d.image + d.sel0_off);
    uint64_t* sel1 = (uint64_t*)(d.image + d.sel1_off);
    if (threadIdx.x == 0) {
        dir[2 * ns] = zeros;
        dir[2 * ns + 1] = 0;
        uint64_t* desc = (uint64_t*)(d.image + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * d.level);
        desc[1] = zeros;
        desc[2] = ones;
    }
    for (uint64_t k = wv_cdiv(ones, WV_SEL_STRIDE) + threadIdx.x; k < d.nsel; k += 256) sel1[k] = d.n;
    for (uint64_t k = wv_cdiv(zeros, WV_SEL_STRIDE) + threadIdx.x; k < d.nsel; k += 256) sel0[k] = d.n;
    uint32_t* sub = (uint32_t*)(d.image + d.sub_off);
    const uint64_t sub_hi = d.nsub - wv_cdiv(zeros, WV_SUB_STRIDE);
    for (uint64_t k = wv_cdiv(ones, WV_SUB_STRIDE) + threadIdx.x; k < sub_hi; k += 256) sub[k] = (uint32_t)d.n;
}

__global__ void __launch_bounds__(256)
b_dir_write_k(const SpanDesc* __restrict__ spans, const uint32_t* __restrict__ chunk0, uint32_t nspan)
{
    // counts and positions of a level fit 32 bits (n < 2^32)
    __shared__ uint32_t wpart[4];
    __shared__ alignas(16) uint32_t zex[SDW];   // zeros of the chunk before each of its words
    __shared__ uint64_t wds[SDW];               // the chunk's words
    const uint32_t s = owner_of(chunk0, nspan, blockIdx.x);
    const SpanDesc& d = spans[s];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n = (uint32_t)d.n, nw = (uint32_t)wv_cdiv(n, 64), ns = (uint32_t)wv_cdiv(n, WV_SB_BITS);
    const uint32_t nch = (uint32_t)wv_cdiv(nw, SDW);
    const uint64_t* words = (const uint64_t*)(d.image + d.bits_off);
    uint64_t* dir = (uint64_t*)(d.image + d.rank_off);
    uint64_t* sel0 = (uint64_t*)(d.image + d.sel0_off);
    uint64_t* sel1 = (uint64_t*)(d.image + d.sel1_off);
    uint32_t* sub = (uint32_t*)(d.image + d.sub_off);
    const uint32_t c0 = (blockIdx.x - d.chunk0) * SDG;
    for (uint32_t c = c0; c < min(nch, c0 + SDG); c++) {   // uniform
        const uint32_t cw = c * SDW, wl = 2 * threadIdx.x, w0 = cw + wl;
        const uint64_t x0 = w0 < nw ? words[w0] : 0ull, x1 = w0 + 1 < nw ? words[w0 + 1] : 0ull;
        const uint32_t cbits = (uint32_t)min<uint64_t>(64ull * cw, n);
        const uint32_t nloc = min(n - cbits, 64u * SDW);    // level bits in the chunk
        const uint32_t obase = (uint32_t)d.pre[c];           // ones before the chunk
        const uint32_t zbase = cbits - obase;
        const uint32_t o0 = __popcll(x0), o1 = __popcll(x1);
        uint32_t tot;
        const uint32_t ex = wave_excl_scan(o0 + o1, &tot);
        if (lane == 0) wpart[wave] = tot;
        __syncthreads();
        uint32_t off = 0, ones = 0;
        for (uint32_t k = 0; k < 4; k++) {
            if (k < wave) off += wpart[k];
            ones += wpart[k];
        }
        const uint32_t ob0 = off + ex, ob1 = ob0 + o0;     // ones of the chunk before my words
        zex[wl] = min(64u * wl, nloc) - ob0;
        zex[wl + 1] = min(64u * (wl + 1), nloc) - ob1;
        wds[wl] = x0;
        wds[wl + 1] = x1;
        __syncthreads();
        // the ones / zeros of ordinal 512k in the chunk: sub-samples, and
        // samples when 4096 divides them
        wv_chunk_samples(wds, zex, min(SDW, nw - cw), nloc, cw, obase, zbase, ones, sub, (uint32_t)d.nsub, sel0, sel1);
        if (threadIdx.x < SDW / 8) {
            const uint32_t k = cw / 8 + threadIdx.x;
            if (k < ns) {
                const uint4 za = *(const uint4*)(zex + 8 * threadIdx.x), zb4 = *(const uint4*)(zex + 8 * threadIdx.x + 4);
                const uint32_t zb = za.x;
                const uint32_t lo = (za.y - zb) | ((za.z - zb) << 9) | ((za.w - zb) << 18);
                const uint32_t hi = (zb4.x - zb) | ((zb4.y - zb) << 9) | ((zb4.z - zb) << 18);
                dir[2 * (uint64_t)k] = zbase + zb;
                dir[2 * (uint64_t)k + 1] = (uint64_t)lo | ((uint64_t)hi << 27) | ((uint64_t)(zb4.w - zb) << 54);
            }
        }
        __syncthreads();   // zex, wds and wpart are rewritten by the next chunk
    }
}

__global__ void __launch_bounds__(256)
b_header_k(uint8_t* const* __restrict__ images, const wv_layout_in* __restrict__ lins, uint32_t count,
           uint32_t* __restrict__ zero, uint64_t nzero)
{
    // the work queues and the histogram area start at zero
    grid_zero(zero, nzero);
    if (blockIdx.x >= count) return;   // whole workgroups; clearing only
    // same header writer as a single build, one workgroup per image
    __shared__ wv_layout_out lay;
    __shared__ uint64_t span_lo[6 * WV_MAX_LEVELS + 4], span_hi[6 * WV_MAX_LEVELS + 4];
    __shared__ int nspan;
    uint8_t* img = images[blockIdx.x];
    const wv_layout_in& in = lins[blockIdx.x];
    if (threadIdx.x == 0) {
        wv_layout(in, lay);
        int s = 0;
        span_lo[s] = 0;
        span_hi[s++] = WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * in.nlevels;
        for (uint32_t l = 0; l < in.nlevels; l++) {
            const wv_level& L = lay.lv[l];
            span_lo[s] = L.bits_off;  span_hi[s++] = L.bits_off + wv_bits_bytes(L.n);
            span_lo[s] = L.rank_off;  span_hi[s++] = L.rank_off + wv_rank_bytes(L.n);
            span_lo[s] = L.sel0_off;  span_hi[s++] = L.sel0_off + 8 * L.nsel;
            span_lo[s] = L.sel1_off;  span_hi[s++] = L.sel1_off + 8 * L.nsel;
            span_lo[s] = L.sub_off;   span_hi[s++] = L.sub_off + 4 * L.nsub;
            span_lo[s] = L.pool_off;  span_hi[s++] = L.pool_off + wv_pool_bytes(L.n);
        }
        span_lo[s] = lay.image_bytes;
        span_hi[s] = lay.image_bytes;
        nspan = s;
        uint32_t* h32 = (uint32_t*)img;
        uint64_t* h64 = (uint64_t*)img;
        h32[0] = WV_MAGIC; h32[1] = WV_VERSION; h32[2] = in.kind; h32[3] = in.arity_log2;
        h64[2] = in.n; h32[6] = in.sigma; h32[7] = in.nlevels; h32[8] = in.key_bits; h32[9] = 0;
        h64[5] = lay.image_bytes; h64[6] = WV_HEADER_BYTES; h64[7] = 0; h64[8] = 0; h64[9] = 0; h64[10] = 0;
    }
    __syncthreads();
    for (uint32_t b = 88 + threadIdx.x; b < WV_HEADER_BYTES; b += blockDim.x) img[b] = 0;
    if (threadIdx.x < in.nlevels) {
        const wv_level& L = lay.lv[threadIdx.x];
        uint64_t* e = (uint64_t*)(img + WV_HEADER_BYTES + (uint64_t)WV_LEVEL_BYTES * threadIdx.x);
        e[0] = L.n; e[1] = 0; e[2] = 0; e[3] = L.bits_off; e[4] = L.rank_off; e[5] = L.sel0_off;
        e[6] = L.sel1_off; e[7] = L.nsel;
    }
    for (int s = 0; s < nspan; s++)
        for (uint64_t b = span_hi[s] + threadIdx.x; b < span_lo[s + 1]; b += blockDim.x) img[b] = 0;
}

// explicit select answers of the long sub-ranges (wv_xsel_block), one
// workgroup per pool slot of every listed level
__global__ void __launch_bounds__(WV_SUB_STRIDE)
b_xsel_k(const wv_xlevel* __restrict__ xs, uint32_t nx)
{
    uint32_t lo = 0, hi = nx - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (xs[mid].blk0 <= blockIdx.x) lo = mid; else hi = mid - 1;
    }
    wv_xsel_block(xs[lo], blockIdx.x - xs[lo].blk0);
}

inline uint32_t width_of(uint32_t bits) { return bits <= 8 ? 1u : (bits <= 16 ? 2u : 4u); }

// ---- host planning -----------------------------------------------------------------

struct SeqPlan {
    uint32_t L, tau, passes, K, C, sym_bytes, sigma;
    uint64_t n;
    uint64_t off_H, off_tot, off_G0, off_pay[2], off_dcnt, off_dpre;
    // image layout: every level of a matrix has n bits, so level l's arrays
    // sit at level 0's offsets + l * lstride
    uint64_t bits0, rank0, sel00, sel10, sub0, pool0, lstride, nsel, nsub, image_bytes;
    wv_level lv(uint32_t l) const
    {
        const uint64_t d = (uint64_t)l * lstride;
        return wv_level{n, bits0 + d, rank0 + d, sel00 + d, sel10 + d, nsel, sub0 + d, nsub, pool0 + d, wv_nslot(n)};
    }
};

// the layout input of a matrix image of n symbols and L levels
inline wv_layout_in matrix_layout_in(uint64_t n, uint32_t sigma, uint32_t L)
{
    wv_layout_in in{};
    in.kind = WT_KIND_WM; in.arity_log2 = 1; in.nlevels = L; in.key_bits = L;
    in.sigma = sigma; in.n = n;
    for (uint32_t l = 0; l < L; l++) in.level_n[l] = n;
    return in;
}

struct BatchPlan {
    std::vector<SeqPlan> seq;
    std::vector<uint32_t> order;     // sequences by decreasing n
    uint64_t off_desc = 0, off_queue = 0, ws_bytes = 0;
    uint64_t zero_lo = 0, zero_hi = 0;   // H region, cleared before every group
    uint32_t max_passes = 0, nphases = 0;
    // descriptor area of every phase (header, every round's two groups, the
    // directories): offset inside the descriptor region and members
    std::vector<uint64_t> phase_off;
    std::vector<uint32_t> phase_members;
    uint64_t desc_total = 0;
};

// most tiles per chunk of a batched build, and the chunks each resident pass
// workgroup should get at least (a sequence's chunk count is also capped at
// the resident pass workgroups, as for one build)
constexpr uint64_t BATCH_CHUNK_TILES = 16;
constexpr uint64_t BATCH_CHUNKS_PER_WORKER = 4;

int make_batch_plan(const wt_seq_desc* seqs, uint32_t count, const wt_tuning* tune, BatchPlan& bp)
{
    bp.seq.resize(count);
    uint64_t off = 0;
    auto bump = [&](uint64_t bytes) { uint64_t at = off; off = wv_round256(off + bytes); return at; };
    // one work-queue counter per phase (at most 2 + 2 * 32 phases), then the
    // histogram areas: the header launch clears both at once
    bp.off_queue = bump(4 * (2 + 2 * 32));
    uint64_t total_chunks = 0, total_spans = 0, total_dch = 0, total_x = 0;
    // One persistent launch serves every sequence, so a chunk can span many
    // tiles: fewer chunks mean fewer histogram workgroups, offset tables and
    // shared boundary words.  Chunks grow only while every pass workgroup
    // still gets about BATCH_CHUNKS_PER_WORKER of them.
    uint64_t total_tiles = 0;
    for (uint32_t i = 0; i < count; i++) total_tiles += wv_cdiv(seqs[i].n ? seqs[i].n : 1, T);
    const uint64_t tiles_per_chunk =
        tune && tune->tile ? tune->tile
                           : std::min<uint64_t>(BATCH_CHUNK_TILES,
                                                std::max<uint64_t>(1, total_tiles / ((uint64_t)KMAX * BATCH_CHUNKS_PER_WORKER)));
    // H of every sequence first (zeroed by one fill every round)
    for (uint32_t i = 0; i < count; i++) {
        const wt_seq_desc& d = seqs[i];
        wt_tuning t1 = tune ? *tune : wt_tuning{};
        if (d.tau) t1.tau = d.tau;
        t1.flags &= ~WT_FLAG_LEVELWISE;
        if (!t1.blocks) t1.blocks = (uint32_t)std::max<uint64_t>(1, wv_cdiv(wv_cdiv(d.n ? d.n : 1, T), tiles_per_chunk));
        t1.tile = 0;
        // the argument checks of wt_plan for a matrix
        if (d.sigma == 0 || (d.sym_bytes != 1 && d.sym_bytes != 2 && d.sym_bytes != 4)) return WT_EINVAL;
        if (d.n >= (1ull << 32)) return WT_EUNSUP;
        wv_wm_plan wp;
        int rc = wv_wm_make_plan(d.n, d.sigma, d.sym_bytes, &t1, wp);
        if (rc) return rc;
        if (!d.S && d.n) return WT_EINVAL;
        if (((uintptr_t)d.S | (uintptr_t)d.out) & 15u) return WT_EINVAL;   // read and written in 16-byte pieces
        SeqPlan& s = bp.seq[i];
        {
            wv_layout_out lay;
            wv_layout(matrix_layout_in(d.n, d.sigma, wp.L), lay);
            s.bits0 = lay.lv[0].bits_off; s.rank0 = lay.lv[0].rank_off;
            s.sel00 = lay.lv[0].sel0_off; s.sel10 = lay.lv[0].sel1_off; s.nsel = lay.lv[0].nsel;
            s.sub0 = lay.lv[0].sub_off; s.nsub = lay.lv[0].nsub; s.pool0 = lay.lv[0].pool_off;
            s.lstride = wp.L > 1 ? lay.lv[1].bits_off - lay.lv[0].bits_off : 0;
            s.image_bytes = lay.image_bytes;
        }
        if (!d.out || d.out_bytes < s.image_bytes) return WT_ENOSPC;
        s.L = wp.L; s.tau = wp.tau; s.K = wp.K; s.C = wp.C; s.n = d.n; s.sym_bytes = d.sym_bytes; s.sigma = d.sigma;
        s.passes = d.n ? (s.L + s.tau - 1) / s.tau : 0;
        bp.max_passes = std::max(bp.max_passes, s.passes);
        s.off_H = bump((uint64_t)256 * s.K * 4);
        total_chunks += s.K;
    }
    bp.zero_lo = bp.seq.empty() ? off : bp.seq[0].off_H;
    bp.zero_hi = off;
    for (uint32_t i = 0; i < count; i++) {
        SeqPlan& s = bp.seq[i];
        s.off_tot = bump(256 * 4);
        s.off_G0 = bump((uint64_t)s.K * MAXG * 4);
        const uint32_t rem = s.L > s.tau ? s.L - s.tau : 0;
        const uint64_t pay = rem ? std::max<uint64_t>(s.n, 1) * width_of(rem) : 0;
        s.off_pay[0] = bump(pay);
        s.off_pay[1] = bump(s.L > 2 * s.tau ? pay : 0);
        const uint64_t dch = wv_cdiv(wv_cdiv(s.n, 64), SDW);
        s.off_dcnt = bump(std::max<uint64_t>(dch, 1) * s.L * 4);
        s.off_dpre = bump(std::max<uint64_t>(dch, 1) * s.L * 8);
        total_spans += s.L;
        total_dch += dch * s.L;
        if (wv_nslot(s.n)) total_x += s.L;
    }
    bp.order.resize(count);
    std::iota(bp.order.begin(), bp.order.end(), 0u);
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](uint32_t a, uint32_t b) { return bp.seq[a].n > bp.seq[b].n; });
    // one descriptor area per phase, each sized for its members, so no phase
    // overwrites descriptors still being read
    bp.nphases = 2 + 2 * bp.max_passes;
    bp.phase_off.assign(bp.nphases + 1, 0);
    bp.phase_members.assign(bp.nphases, 0);
    auto area = [&](uint32_t ph, uint64_t bytes) {
        bp.phase_off[ph] = bp.desc_total;
        bp.desc_total += wv_round256(bytes);
    };
    area(0, wv_round256(count * sizeof(uint8_t*)) + count * sizeof(wv_layout_in));
    for (uint32_t r = 0; r < bp.max_passes; r++) {
        for (int wide = 0; wide < 2; wide++) {
            const uint32_t ph = 1 + 2 * r + wide;
            uint32_t m = 0;
            for (uint32_t i = 0; i < count; i++) {
                const SeqPlan& sp = bp.seq[i];
                if (r < sp.passes && ((sp.L - r * sp.tau > 16) == (wide == 1))) m++;
            }
            bp.phase_members[ph] = m;
            area(ph, wv_round256((uint64_t)m * sizeof(SeqRound)) + wv_round256((uint64_t)m * 4) + (uint64_t)m * 4);
        }
    }
    area(bp.nphases - 1, wv_round256(total_spans * sizeof(SpanDesc)) + wv_round256(total_spans * 4) +
                             total_x * sizeof(wv_xlevel));
    bp.phase_off[bp.nphases] = bp.desc_total;
    bp.off_desc = bump(bp.desc_total);
    bp.ws_bytes = off;
    if (wv_trace_on())
        wv_trace("batch plan: %u sequences, %llu tiles, %llu tiles per chunk, %llu chunks, %u rounds, "
                 "descriptors=%llu workspace=%llu", count, (unsigned long long)total_tiles,
                 (unsigned long long)tiles_per_chunk, (unsigned long long)total_chunks, bp.max_passes,
                 (unsigned long long)bp.desc_total, (unsigned long long)bp.ws_bytes);
    (void)total_dch;
    return WT_OK;
}

}  // namespace

extern "C" {

int wt_batch_plan(int kind, const wt_seq_desc* seqs, uint32_t count, const wt_tuning* tune,
                  uint64_t* workspace_bytes)
{
    if (kind != WT_KIND_WM || (!seqs && count) || !workspace_bytes) return WT_EINVAL;
    BatchPlan bp;
    int rc = make_batch_plan(seqs, count, tune, bp);
    if (rc) return rc;
    *workspace_bytes = bp.ws_bytes;
    return WT_OK;
}

int wt_batch_build(int kind, const wt_seq_desc* seqs, uint32_t count, void* ws_, size_t ws_bytes,
                   const wt_tuning* tune, void* stream)
{
    if (kind != WT_KIND_WM || (!seqs && count)) return WT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    BatchPlan bp;
    int rc = make_batch_plan(seqs, count, tune, bp);
    if (rc) return rc;
    if (!count) return WT_OK;
    if (!ws_ || ws_bytes < bp.ws_bytes) return WT_ENOSPC;
    if ((uintptr_t)ws_ & 15u) return WT_EINVAL;
    uint8_t* ws = (uint8_t*)ws_;
    const bool prof = tune && (tune->flags & WT_FLAG_PROFILE);

    // every descriptor of the build, in one pinned host buffer with an area
    // per phase, all written before the first launch
    PinnedBuf pin(bp.desc_total, s);
    std::vector<uint8_t> unpinned(pin.get() ? 0 : bp.desc_total);
    uint8_t* hd = pin.get() ? (uint8_t*)pin.get() : unpinned.data();
    auto host_area = [&](uint32_t ph) { return hd + bp.phase_off[ph]; };
    auto dev_area = [&](uint32_t ph) { return ws + bp.off_desc + bp.phase_off[ph]; };
    std::memset(hd, 0, bp.desc_total);

    // phase 0: headers of every image
    {
        uint8_t** imgs = (uint8_t**)host_area(0);
        wv_layout_in* lins = (wv_layout_in*)(host_area(0) + wv_round256(count * sizeof(uint8_t*)));
        for (uint32_t i = 0; i < count; i++) {
            imgs[i] = (uint8_t*)seqs[i].out;
            lins[i] = matrix_layout_in(bp.seq[i].n, bp.seq[i].sigma, bp.seq[i].L);
        }
    }
    // rounds of passes: two groups per round, keys up to 16 bits (16-bit LDS
    // keys) and wider ones
    struct Group { uint32_t phase, m, chunks, cols; bool wide; };
    std::vector<Group> groups;
    {
        std::vector<const void*> cur_in(count);
        std::vector<uint32_t> cur_bytes(count);
        for (uint32_t i = 0; i < count; i++) { cur_in[i] = seqs[i].S; cur_bytes[i] = seqs[i].sym_bytes; }
        uint32_t phase = 1;
        for (uint32_t r = 0; r < bp.max_passes; r++) {
            for (int wide = 0; wide < 2; wide++, phase++) {
                std::vector<uint32_t> members;
                for (uint32_t i : bp.order) {
                    const SeqPlan& sp = bp.seq[i];
                    if (r >= sp.passes) continue;
                    const uint32_t R = sp.L - r * sp.tau;
                    if ((R > 16) != (wide == 1)) continue;
                    members.push_back(i);
                }
                if (members.empty()) continue;
                const uint32_t m = (uint32_t)members.size();
                if (m != bp.phase_members[phase]) {   // the plan and the build disagree
                    pin.idle();   // nothing was queued
                    return WT_EINVAL;
                }
                SeqRound* q = (SeqRound*)host_area(phase);
                uint32_t* first = (uint32_t*)(host_area(phase) + wv_round256((uint64_t)m * sizeof(SeqRound)));
                uint32_t* cfirst = first + wv_round256((uint64_t)m * 4) / 4;
                uint32_t chunks = 0, cols = 0;
                for (uint32_t k = 0; k < m; k++) {
                    const uint32_t i = members[k];
                    const SeqPlan& sp = bp.seq[i];
                    const uint32_t l0 = r * sp.tau, tau = std::min(sp.tau, sp.L - l0), R = sp.L - l0, rem = R - tau;
                    SeqRound& e = q[k];
                    e.pa.in = cur_in[i];
                    e.pa.pay_out = rem ? (void*)(ws + sp.off_pay[r & 1]) : nullptr;
                    for (uint32_t j = 0; j < tau; j++)
                        e.pa.words[j] = (uint64_t*)((uint8_t*)seqs[i].out + sp.lv(l0 + j).bits_off);
                    e.pa.G0 = (const uint32_t*)(ws + sp.off_G0);
                    e.pa.n = (uint32_t)sp.n; e.pa.C = sp.C; e.pa.K = sp.K; e.pa.R = R; e.pa.tau = tau;
                    e.pa.keymask = r == 0 ? (sp.L >= 32 ? ~0u : ((1u << sp.L) - 1u)) : ~0u;
                    e.H = (uint32_t*)(ws + sp.off_H);
                    e.tot = (uint32_t*)(ws + sp.off_tot);
                    e.status = r == 0 ? (uint32_t*)((uint8_t*)seqs[i].out + 36) : nullptr;
                    e.in_bytes = cur_bytes[i];
                    e.out_bytes = rem ? width_of(rem) : 1;
                    e.pa.in_bytes = e.in_bytes;
                    e.pa.out_bytes = e.out_bytes;
                    e.sigma = sp.sigma;
                    e.chunk0 = chunks;
                    first[k] = chunks;
                    chunks += sp.K;
                    e.col0 = cols;
                    cfirst[k] = cols;
                    cols += 1u << tau;
                    if (e.pa.pay_out) { cur_in[i] = e.pa.pay_out; cur_bytes[i] = e.out_bytes; }
                }
                groups.push_back(Group{phase, m, chunks, cols, wide == 1});
            }
        }
    }
    // last phase: the directories of every level of every sequence
    const uint32_t dphase = bp.nphases - 1;
    uint32_t nspan = 0, dchunks = 0;   // dchunks: directory workgroups (SDG chunks each)
    uint32_t nx = 0, xblocks = 0;      // levels with pool slots, their workgroups
    {
        for (uint32_t i = 0; i < count; i++) nspan += bp.seq[i].L;
        SpanDesc* sd = (SpanDesc*)host_area(dphase);
        uint32_t* first = (uint32_t*)(host_area(dphase) + wv_round256((uint64_t)nspan * sizeof(SpanDesc)));
        wv_xlevel* xl = (wv_xlevel*)((uint8_t*)first + wv_round256((uint64_t)nspan * 4));
        uint32_t k = 0;
        for (uint32_t i = 0; i < count; i++) {
            const SeqPlan& sp = bp.seq[i];
            const uint64_t dch = wv_cdiv(wv_cdiv(sp.n, 64), SDW);
            for (uint32_t l = 0; l < sp.L; l++, k++) {
                SpanDesc& d = sd[k];
                d.image = (uint8_t*)seqs[i].out;
                d.n = sp.n;
                const wv_level lvl = sp.lv(l);
                d.bits_off = lvl.bits_off;
                d.rank_off = lvl.rank_off;
                d.sel0_off = lvl.sel0_off;
                d.sel1_off = lvl.sel1_off;
                d.nsel = lvl.nsel;
                d.sub_off = lvl.sub_off;
                d.nsub = lvl.nsub;
                d.cnt = (uint32_t*)(ws + sp.off_dcnt) + l * std::max<uint64_t>(dch, 1);
                d.pre = (uint64_t*)(ws + sp.off_dpre) + l * std::max<uint64_t>(dch, 1);
                d.level = l;
                d.chunk0 = dchunks;
                first[k] = dchunks;
                dchunks += (uint32_t)wv_cdiv(dch, SDG);
                if (lvl.nslot) {
                    wv_xlevel& x = xl[nx++];
                    x.image = d.image;
                    x.m = sp.n;
                    x.bits_off = lvl.bits_off;
                    x.rank_off = lvl.rank_off;
                    x.sub_off = lvl.sub_off;
                    x.nsub = lvl.nsub;
                    x.blk0 = xblocks;
                    xblocks += (uint32_t)(2 * lvl.nslot);
                }
            }
        }
    }

    // nothing has been launched before this point: every error above leaves
    // the stream untouched
    WV_TIMED(prof, s, "b_desc_copy",
             WV_CHECK(pin.get() ? wv_upload(ws + bp.off_desc, hd, bp.desc_total, s)
                                : hipMemcpyAsync(ws + bp.off_desc, hd, bp.desc_total, hipMemcpyHostToDevice, s)));
    uint32_t* hzero = (uint32_t*)(ws + bp.zero_lo);
    const uint64_t nhzero = (bp.zero_hi - bp.zero_lo) / 4;
    {
        const uint64_t nz = (bp.zero_hi - bp.off_queue) / 4;
        const uint32_t zb = (uint32_t)std::min<uint64_t>(wv_cdiv(nz, 256 * 16), 4096);
        WV_TIMED(prof, s, "b_header",
                 (b_header_k<<<count + zb, 256, 0, s>>>((uint8_t* const*)dev_area(0),
                                                        (const wv_layout_in*)(dev_area(0) + wv_round256(count * sizeof(uint8_t*))),
                                                        count, (uint32_t*)(ws + bp.off_queue), nz)));
        WV_CHECK(hipGetLastError());
    }
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const Group& g = groups[gi];
        uint8_t* desc = dev_area(g.phase);
        const SeqRound* dq = (const SeqRound*)desc;
        const uint32_t* dfirst = (const uint32_t*)(desc + wv_round256((uint64_t)g.m * sizeof(SeqRound)));
        const uint32_t* dcfirst = dfirst + wv_round256((uint64_t)g.m * 4) / 4;
        uint32_t* queue = (uint32_t*)(ws + bp.off_queue) + g.phase;
        // the last group leaves the histogram area as it is
        const uint64_t nz = gi + 1 < groups.size() ? nhzero : 0;
        WV_TIMED(prof, s, "b_hist", (b_hist_k<<<g.chunks * HSPLIT, HT, 0, s>>>(dq, dfirst, g.m)));
        WV_TIMED(prof, s, "b_scan", (b_scan_k<<<wv_cdiv(g.cols, HT / 64), HT, 0, s>>>(dq, dcfirst, g.m, g.cols)));
        WV_TIMED(prof, s, "b_offsets", (b_offsets_k<<<g.chunks, HT, 0, s>>>(dq, dfirst, g.m)));
        const uint32_t workers = std::min<uint32_t>(g.chunks, g.wide ? KRES32 : KRES16);
        WV_TIMED(prof, s, "b_pass",
                 (g.wide ? (void)(b_pass32_k<<<workers, NT, 0, s>>>(dq, dfirst, g.m, g.chunks, queue, hzero, nz))
                         : (void)(b_pass16_k<<<workers, NT, 0, s>>>(dq, dfirst, g.m, g.chunks, queue, hzero, nz))));
        WV_CHECK(hipGetLastError());
    }
    {
        uint8_t* desc = dev_area(dphase);
        const SpanDesc* dsd = (const SpanDesc*)desc;
        const uint32_t* dfirst = (const uint32_t*)(desc + wv_round256((uint64_t)nspan * sizeof(SpanDesc)));
        if (dchunks) WV_TIMED(prof, s, "b_dir_count", (b_dir_count_k<<<dchunks, 256, 0, s>>>(dsd, dfirst, nspan)));
        WV_TIMED(prof, s, "b_dir_scan", (b_dir_scan_k<<<nspan, 256, 0, s>>>(dsd)));
        if (dchunks) WV_TIMED(prof, s, "b_dir_write", (b_dir_write_k<<<dchunks, 256, 0, s>>>(dsd, dfirst, nspan)));
        const wv_xlevel* dxl = (const wv_xlevel*)((const uint8_t*)dfirst + wv_round256((uint64_t)nspan * 4));
        if (xblocks) WV_TIMED(prof, s, "b_dir_explicit", (b_xsel_k<<<xblocks, WV_SUB_STRIDE, 0, s>>>(dxl, nx)));
        WV_CHECK(hipGetLastError());
    }
    // the upload reads the host descriptors: the pinned buffer returns to the
    // pool once the stream is past it (a pageable fallback, used only when no
    // pinned memory could be had, must be waited for)
    if (pin.get()) pin.retire(s);
    else WV_CHECK(hipStreamSynchronize(s));
    return WT_OK;
}

}  // extern "C"
