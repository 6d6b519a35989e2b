// wv_wm_core.h -- device code of the wavelet-matrix partition passes, shared
// by the single build (wv_wm_passes.hip) and the batched build
// (wv_batch.hip).  See wv_wm_passes.hip for the method.
#pragma once

#include "wv_internal.h"

namespace {

constexpr int NT = 512;             // threads of a pass workgroup
constexpr int NWAVE = NT / 64;
constexpr int E = 16;               // elements per thread per tile
constexpr int T = NT * E;           // tile
constexpr int TW = T / 64;          // bit words per tile level
constexpr int MAXG = 511;           // run groups of sub-levels j = 0..8
constexpr int HT = 256;             // histogram / scan threads
// resident pass workgroups on the 256 CUs: four per CU (8 waves per SIMD
// within 64 VGPRs) with 16-bit keys in LDS, three with 32-bit keys (LDS-bound)
constexpr uint32_t KRES16 = 1024;
constexpr uint32_t KRES32 = 768;
constexpr uint32_t KMAX = KRES16;    // most chunks of one build by default
// bytes of the word -> run table of a sub-level (TW words plus one partial
// word for each of at most 128 runs), a multiple of 256: WRW words per lane
constexpr uint32_t WRB = (TW + 128 + 255) / 256 * 256;
constexpr uint32_t WRW = WRB / 256;


__device__ __host__ inline uint32_t gidx(uint32_t j, uint32_t u) { return (1u << j) - 1u + u; }

__device__ inline uint32_t brev(uint32_t v, uint32_t nbits) { return nbits ? (__brev(v) >> (32 - nbits)) : 0u; }

struct PassArgs {
    const void* in;
    void* pay_out;
    uint64_t* words[8];     // bit arrays of levels a*tau + j
    const uint32_t* G0;     // [K][MAXG] first run offset of every chunk
    uint32_t n, C, K;       // elements, chunk length (multiple of T), chunks
    uint32_t R, tau;        // key bits still to do, digit bits of this pass
    uint32_t keymask;       // applied to the loaded keys
    uint32_t in_bytes;      // width of the input keys (1, 2, 4)
    uint32_t out_bytes;     // width of the compacted remaining keys written (1, 2, 4)
};

template <typename T_>
__device__ inline uint32_t ld(const void* p, uint64_t i) { return (uint32_t)((const T_*)p)[i]; }

// 64 bits of the tile bit string starting at bit `src`, keeping `nb` (1..64)
__device__ inline uint64_t extract(const uint64_t* lb, uint32_t src, uint32_t nb)
{
    const uint32_t w = src >> 6, o = src & 63;
    uint64_t v = lb[w] >> o;
    if (o && o + nb > 64) v |= lb[w + 1] << (64 - o);
    return nb >= 64 ? v : (v & ((1ull << nb) - 1ull));
}

__device__ inline uint64_t lanemask_lt()
{
    const uint32_t lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// exclusive scan of the 64 values held by one wave (lane l holds v); every
// lane must be active
__device__ inline uint32_t wave_excl_scan(uint32_t v, uint32_t* total)
{
    const uint32_t inc = wv_wave_incl_scan(v);
    *total = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    return inc - v;
}

// inclusive max-scan of the 64 values held by one wave (every lane active)
__device__ inline uint32_t wave_incl_max(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));   // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));   // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));   // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));   // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return v;
}

// LDS writes of this wave visible to its other lanes
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename IT, typename KT_>
__device__ inline void load_tile(const void* in, uint32_t ts, uint32_t tc, uint32_t keymask, KT_* buf)
{
    // 16-byte loads; tile starts are multiples of the tile, so aligned
    constexpr uint32_t V = 16 / sizeof(IT);
    const uint32_t nv = tc / V;
    const uint4* src = (const uint4*)((const IT*)in + ts);
    if (tc == (uint32_t)T) {
        // a whole tile: every load of the thread in flight at once
        constexpr uint32_t NV = T / V / NT;
        uint4 qs[NV];
        for (uint32_t u = 0; u < NV; u++) qs[u] = src[threadIdx.x + u * NT];
        for (uint32_t u = 0; u < NV; u++) {
            const uint32_t v = threadIdx.x + u * NT;
            const uint32_t wd[4] = {qs[u].x, qs[u].y, qs[u].z, qs[u].w};
            for (uint32_t k = 0; k < V; k++) {
                const uint32_t x = (sizeof(IT) == 4) ? wd[k]
                                 : (sizeof(IT) == 2) ? ((wd[k / 2] >> (16 * (k & 1))) & 0xFFFFu)
                                                     : ((wd[k / 4] >> (8 * (k & 3))) & 0xFFu);
                buf[v * V + k] = (KT_)(x & keymask);
            }
        }
        return;
    }
    for (uint32_t v = threadIdx.x; v < nv; v += NT) {
        const uint4 q = src[v];
        const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
        for (uint32_t k = 0; k < V; k++) {
            const uint32_t x = (sizeof(IT) == 4) ? wd[k]
                             : (sizeof(IT) == 2) ? ((wd[k / 2] >> (16 * (k & 1))) & 0xFFFFu)
                                                 : ((wd[k / 4] >> (8 * (k & 3))) & 0xFFu);
            buf[v * V + k] = (KT_)(x & keymask);
        }
    }
    for (uint32_t p = nv * V + threadIdx.x; p < tc; p += NT) buf[p] = (KT_)(ld<IT>(in, (uint64_t)ts + p) & keymask);
    // a partial tile is padded with keys whose every bit is one: on every
    // sub-level they are ones behind all real ones, so they stay at the end
    for (uint32_t p = tc + threadIdx.x; p < (uint32_t)T; p += NT) buf[p] = (KT_)~0u;
}

// the tile's keys from input of any width (a switch per tile: the kernels
// hold one copy of the pass for every width)
template <typename KT_>
__device__ inline void load_tile_any(const void* in, uint32_t in_bytes, uint32_t ts, uint32_t tc, uint32_t keymask,
                                     KT_* buf)
{
    if (in_bytes == 1) load_tile<uint8_t, KT_>(in, ts, tc, keymask, buf);
    else if (in_bytes == 2) load_tile<uint16_t, KT_>(in, ts, tc, keymask, buf);
    else load_tile<uint32_t, KT_>(in, ts, tc, keymask, buf);
}

// zeros among the first s bits of the tile bit string (s <= tile length)
__device__ inline uint32_t local_rank0(const uint64_t* lb, const uint32_t* zw, uint32_t s)
{
    const uint32_t w = s >> 6, o = s & 63;
    uint32_t z = zw[w];
    if (o) z += o - __popcll(lb[w] & ((1ull << o) - 1ull));
    return z;
}

// LDS of one pass workgroup; KT_ holds the keys (16 bits when at most 16
// key bits remain)
template <typename KT_>
struct PassShared {
    KT_ buf[T];
    uint64_t lb[TW + 1];
    uint32_t zw[TW + 1];
    alignas(16) uint32_t zt[TW];   // zw of word e * NWAVE + w at zt[w * E + e]
    uint32_t cnt[MAXG], ls[MAXG], g[MAXG], fw[MAXG];
    uint64_t carry[2][255];
    uint32_t sp[129];
    // run (index inside its sub-level) owning each word a sub-level writes:
    // at most TW words plus one partial word per run (runs of one sub-level
    // number at most 128)
    alignas(16) uint8_t wr[WRB];
};

// One chunk b of one pass (see the file comment of wv_wm_passes.hip).
template <typename KT_>
__device__ void wm_pass_chunk(const PassArgs& a, uint32_t b, PassShared<KT_>& S)
{
    KT_* buf = S.buf;
    uint64_t* lb = S.lb;
    uint32_t* zw = S.zw;
    uint32_t *cnt = S.cnt, *ls = S.ls, *g = S.g, *fw = S.fw;
    uint64_t (*carry)[255] = S.carry;
    uint32_t* sp = S.sp;

    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t tau = a.tau, R = a.R;
    const uint32_t ngroups = (2u << tau) - 1u;         // j = 0..tau
    // chunk b starts below n (< 2^32); its end is taken in 64 bits, as the
    // chunks together may cover 2^32 keys or more
    const uint32_t cstart = b * a.C;
    const uint32_t cend = (uint32_t)min<uint64_t>(a.n, (uint64_t)cstart + a.C);
    const uint32_t ntiles = (cend - cstart + (uint32_t)T - 1) / (uint32_t)T;
    const uint32_t dshift = R - tau;
    const uint32_t dmask = (1u << tau) - 1u;
    const uint32_t pmask = dshift >= 32 ? ~0u : ((1u << dshift) - 1u);

    for (uint32_t i = tid; i < ngroups; i += NT) {
        const uint32_t g0 = a.G0[(uint64_t)b * MAXG + i];
        g[i] = g0;
        fw[i] = (g0 & 63u) ? (g0 >> 6) : 0xFFFFFFFFu;
        if (i < 255) carry[0][i] = 0;
    }
    if (tid == 0) lb[TW] = 0;
    uint32_t cpar = 0;   // carry buffer read this tile

    for (uint32_t tile = 0; tile < ntiles; tile++) {   // no tile start wraps past 2^32
        const uint32_t ts = cstart + tile * (uint32_t)T;
        const uint32_t tc = min((uint32_t)T, cend - ts);
        load_tile_any<KT_>(a.in, a.in_bytes, ts, tc, a.keymask, buf);
        if (tid == 0) { cnt[0] = tc; ls[0] = 0; }
        __syncthreads();

        for (uint32_t j = 0; j < tau; j++) {
            // phase 1: bit j of every element, in the order of sub-level j
            // (one ballot word per 64 elements)
            uint32_t xs[E];
            uint64_t balls[E];
            bool bit[E];
            const uint32_t sh = R - 1 - j;
            for (int e = 0; e < E; e++) xs[e] = (uint32_t)buf[tid + NT * e];
            for (int e = 0; e < E; e++) {
                bit[e] = (xs[e] >> sh) & 1u;
                balls[e] = __ballot(bit[e]);
            }
            if (lane == 0)
                for (int e = 0; e < E; e++) lb[e * NWAVE + wave] = balls[e];
            const uint32_t nk = 1u << j;
            const uint32_t gb = gidx(j, 0);
            __syncthreads();
            // phase 2: zero prefix over the words (wave 0), run slots (wave 1)
            if (wave == 0) {
                uint32_t v[TW / 64];
                for (uint32_t k = 0; k < TW / 64; k++) v[k] = 64u - (uint32_t)__popcll(lb[64 * k + lane]);
                uint32_t run = 0;
                for (uint32_t k = 0; k < TW / 64; k++) {
                    uint32_t tot;
                    const uint32_t ex = wave_excl_scan(v[k], &tot);
                    zw[64 * k + lane] = run + ex;
                    {
                        const uint32_t w = 64 * k + lane;
                        S.zt[(w % NWAVE) * E + w / NWAVE] = run + ex;
                    }
                    run += tot;
                }
                if (lane == 0) zw[TW] = run;
            } else if (wave == 1) {
                // words every run of sub-level j completes in this tile, their
                // prefix, and the run owning each of those words: a run's
                // first word marks its index, and a forward max over the
                // table fills the words after it (run indices increase)
                uint32_t* wr4 = (uint32_t*)S.wr;
                for (uint32_t k = 0; k < WRW; k++) wr4[WRW * lane + k] = 0;
                wave_lds_sync();
                uint32_t run = 0;
                for (uint32_t u0 = 0; u0 < nk; u0 += 64) {
                    const uint32_t u = u0 + lane;
                    uint32_t v = 0;
                    if (u < nk) {
                        const uint32_t gg = g[gb + u];
                        v = ((gg + cnt[gb + u]) >> 6) - (gg >> 6);
                    }
                    uint32_t tot;
                    const uint32_t ex = wave_excl_scan(v, &tot);
                    if (u < nk) {
                        sp[u] = run + ex;
                        if (v) S.wr[run + ex] = (uint8_t)u;
                    }
                    run += tot;
                }
                if (lane == 0) sp[nk] = run;
                wave_lds_sync();
                uint32_t q[WRW], m = 0;
                for (uint32_t k = 0; k < WRW; k++) {
                    q[k] = wr4[WRW * lane + k];
                    for (uint32_t b = 0; b < 4; b++) {     // forward max inside the lane's bytes
                        m = max(m, (q[k] >> (8 * b)) & 0xFFu);
                        q[k] = (q[k] & ~(0xFFu << (8 * b))) | (m << (8 * b));
                    }
                }
                const uint32_t incl = wave_incl_max(m);
                const uint32_t prev = (uint32_t)__shfl_up((int)incl, 1);
                const uint32_t ex = lane ? prev : 0u;
                for (uint32_t k = 0; k < WRW; k++) {
                    uint32_t r = 0;
                    for (uint32_t b = 0; b < 4; b++) r |= max(ex, (q[k] >> (8 * b)) & 0xFFu) << (8 * b);
                    wr4[WRW * lane + k] = r;
                }
            }
            __syncthreads();
            // phase 3: partition, child runs, emit words
            const uint32_t ztot = zw[TW];
            // every element moves to its place in the order of sub-level
            // j+1 (padding keys are ones on every sub-level and stay in
            // place); the last sub-level's order is needed only for the
            // payload of the next pass
            if (j + 1 < tau || a.pay_out) {
                const uint4* zt4 = (const uint4*)(S.zt + wave * E);
#pragma unroll
                for (int q = 0; q < E / 4; q++) {
                    const uint4 z4 = zt4[q];
                    const uint32_t zz[4] = {z4.x, z4.y, z4.z, z4.w};
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int e = 4 * q + u;
                        const uint32_t p = tid + NT * e;
                        // zeros before the element in the tile: its word's
                        // prefix plus the zeros of lower lanes (mbcnt adds
                        // its count to the prefix)
                        const uint64_t nb = ~balls[e];
                        const uint32_t zb = __builtin_amdgcn_mbcnt_hi((uint32_t)(nb >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)nb, zz[u]));
                        buf[bit[e] ? ztot + (p - zb) : zb] = (KT_)xs[e];
                    }
                }
            }
            // runs of sub-level j+1 split the runs of j by bit j; a child's
            // elements keep their order, zeros of the tile first
            const uint32_t gc = gidx(j + 1, 0);
            uint64_t* words = a.words[j];
            // child runs on the last threads, words on the threads after the
            // first two waves (which did the scans of this sub-level)
            for (uint32_t u = NT - 1 - tid; u < nk; u += NT) {
                const uint32_t s0 = ls[gb + u], c = cnt[gb + u];
                const uint32_t zs = local_rank0(lb, zw, s0), ze = local_rank0(lb, zw, s0 + c);
                cnt[gc + 2 * u] = ze - zs;
                cnt[gc + 2 * u + 1] = c - (ze - zs);
                ls[gc + 2 * u] = zs;
                ls[gc + 2 * u + 1] = ztot + (s0 - zs);
                // the partial last word of the run, carried to the next tile
                const uint32_t gi = gb + u;
                const uint32_t gg = g[gi], en = gg + c;
                uint64_t v = 0;
                if (en & 63u) {
                    const uint32_t We = en >> 6;
                    const uint32_t wlo = max(We * 64u, gg);
                    const uint32_t nb = en - wlo;
                    if (nb) v = extract(lb, s0 + (wlo - gg), nb) << (wlo - We * 64u);
                    if (We == (gg >> 6)) v |= carry[cpar][gi];
                }
                carry[cpar ^ 1][gi] = v;
            }
            const uint32_t total = sp[nk];
            for (uint32_t s = (tid + NT - 128) % NT; s < total; s += NT) {
                const uint32_t lo = S.wr[s];
                const uint32_t gi = gb + lo;
                const uint32_t i = s - sp[lo];
                const uint32_t gg = g[gi];
                const uint32_t W = (gg >> 6) + i;
                const uint32_t wlo = max(W * 64u, gg);
                const uint32_t nb = W * 64u + 64u - wlo;
                uint64_t v = extract(lb, ls[gi] + (wlo - gg), nb) << (wlo - W * 64u);
                if (i == 0) v |= carry[cpar][gi];
                if (W == fw[gi]) atomicOr((unsigned long long*)&words[W], (unsigned long long)v);
                else words[W] = v;
            }
            __syncthreads();
        }
        // remaining key bits to the order of the next pass
        if (a.pay_out) {
            const uint32_t ob = a.out_bytes;
            for (int e = 0; e < E; e++) {
                const uint32_t p = tid + NT * e;
                if (p < tc) {
                    const uint32_t x = buf[p];
                    const uint32_t gi = gidx(tau, (x >> dshift) & dmask);
                    const uint32_t at = g[gi] + (p - ls[gi]);
                    if (ob == 1) ((uint8_t*)a.pay_out)[at] = (uint8_t)(x & pmask);
                    else if (ob == 2) ((uint16_t*)a.pay_out)[at] = (uint16_t)(x & pmask);
                    else ((uint32_t*)a.pay_out)[at] = x & pmask;
                }
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < ngroups; i += NT) g[i] += cnt[i];
        cpar ^= 1;
        __syncthreads();
    }
    // flush the partial words left at the end of the chunk
    for (uint32_t i = tid; i < (1u << tau) - 1u; i += NT) {
        const uint32_t j = 31 - __clz(i + 1);
        if ((g[i] & 63u) && carry[cpar][i])
            atomicOr((unsigned long long*)&a.words[j][g[i] >> 6], (unsigned long long)carry[cpar][i]);
    }
}

constexpr uint32_t HSPLIT = 2;       // histogram workgroups per chunk
constexpr uint32_t HUNROLL = 4;      // 16-byte loads in flight per thread
// LDS histograms of a workgroup: HCOPY per wave, lane l adding into copy
// l % HCOPY, so that lanes holding the same frequent digit seldom hit one
// address in one atomic; copies HSTRIDE words apart put a bin's copies in
// different banks
constexpr uint32_t HCOPY = 4;
constexpr uint32_t HSTRIDE = 257;
constexpr uint32_t HWORDS = (HT / 64) * HCOPY * HSTRIDE;

__device__ inline uint32_t sym_of(const uint32_t* wds, uint32_t k, uint32_t size)
{
    return size == 4 ? wds[k] : (size == 2 ? ((wds[k / 2] >> (16 * (k & 1))) & 0xFFFFu)
                                           : ((wds[k / 4] >> (8 * (k & 3))) & 0xFFu));
}

// per-chunk histogram of the pass digit (first pass: also validates S);
// HSPLIT workgroups share a chunk and add their counts into H
template <typename IT>
__device__ void wm_hist_part(const void* __restrict__ in, uint32_t n, uint32_t C, uint32_t K, uint32_t R,
                             uint32_t tau, uint32_t keymask, uint32_t* __restrict__ H,
                             uint32_t* __restrict__ status, uint32_t sigma, uint32_t b, uint32_t part,
                             uint32_t* h)
{
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t cs = b * C, ce = (uint32_t)min<uint64_t>(n, (uint64_t)cs + C);
    const uint32_t dshift = R - tau, dmask = (1u << tau) - 1u;
    for (uint32_t i = threadIdx.x; i < HWORDS; i += HT) h[i] = 0;
    uint32_t* hw = h + (wave * HCOPY + (threadIdx.x & (HCOPY - 1))) * HSTRIDE;
    __syncthreads();
    bool bad = false;
    constexpr uint32_t V = 16 / sizeof(IT);
    // the chunk's 16-byte vectors (chunk starts are tile multiples, so
    // aligned), split evenly over the HSPLIT workgroups
    const uint32_t nvec = (ce - cs) / V;
    const uint32_t per = (nvec + HSPLIT - 1) / HSPLIT;
    const uint32_t vs = cs / V + part * per;
    const uint32_t ve = cs / V + min(nvec, (part + 1) * per);
    const uint4* in4 = (const uint4*)in;
    for (uint32_t v0 = vs + threadIdx.x; v0 < ve; v0 += HT * HUNROLL) {
        uint4 q[HUNROLL];
        for (uint32_t u = 0; u < HUNROLL; u++) {
            const uint32_t v = v0 + u * HT;
            q[u] = v < ve ? in4[v] : make_uint4(0, 0, 0, 0);
        }
        for (uint32_t u = 0; u < HUNROLL; u++) {
            if (v0 + u * HT >= ve) break;
            const uint32_t wds[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
            // runs of equal digits (common once the sequence is grouped by
            // its leading bits) are added at once
            uint32_t cur = ((sym_of(wds, 0, sizeof(IT)) & keymask) >> dshift) & dmask, run = 0;
            for (uint32_t k = 0; k < V; k++) {
                const uint32_t x = sym_of(wds, k, sizeof(IT));
                bad |= x >= sigma;
                const uint32_t d = ((x & keymask) >> dshift) & dmask;
                if (d != cur) {
                    atomicAdd(&hw[cur], run);
                    cur = d;
                    run = 0;
                }
                run++;
            }
            atomicAdd(&hw[cur], run);
        }
    }
    if (part == HSPLIT - 1) {
        // 64-bit index: ce may lie within HT of 2^32
        for (uint64_t i = (uint64_t)cs + nvec * V + threadIdx.x; i < ce; i += HT) {
            const uint32_t x = ld<IT>(in, i);
            bad |= x >= sigma;
            atomicAdd(&hw[((x & keymask) >> dshift) & dmask], 1u);
        }
    }
    if (status && __ballot(bad) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, 1u);
    __syncthreads();
    if (threadIdx.x <= dmask) {
        uint32_t c = 0;
        for (uint32_t k = 0; k < (HT / 64) * HCOPY; k++) c += h[k * HSTRIDE + threadIdx.x];
        if (c) atomicAdd(&H[(uint64_t)threadIdx.x * K + b], c);
    }
}

// exclusive prefix of every digit's counts over the chunks (in place)
__global__ void __launch_bounds__(HT)
wm_scan_chunks_k(uint32_t* __restrict__ H, uint32_t K, uint32_t* __restrict__ totals)
{
    __shared__ uint32_t ws[HT / 64];
    const uint32_t d = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t* h = H + (uint64_t)d * K;
    uint32_t run = 0;
    for (uint32_t base = 0; base < K; base += HT) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < K ? h[i] : 0u;
        uint32_t wt;
        const uint32_t ex = wave_excl_scan(v, &wt);
        if (lane == 0) ws[wave] = wt;
        __syncthreads();
        uint32_t off = 0, tot = 0;
        for (uint32_t w = 0; w < HT / 64; w++) {
            if (w < wave) off += ws[w];
            tot += ws[w];
        }
        if (i < K) h[i] = run + off + ex;
        run += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[d] = run;
}

// Run offsets of one chunk.  Run (j, u) holds the keys whose top j digit
// bits are u on sub-level j of the pass; its start on the level is the total
// of the runs before it in bit-reversed key order, and chunk b's part of it
// starts after the run's keys of the chunks before b.  On entry cj[gidx(tau,
// d)] holds digit d's count in the chunks before b and tj[gidx(tau, d)] its
// total, for every d < 2^tau; the coarser runs are sums of their two halves.
struct OffShared {
    uint32_t cj[MAXG], tj[MAXG], bs[MAXG];
};

// natural: runs in key order (the tree order of a balanced tree's level,
// Sec. 2) instead of the matrix's bit-reversed order (Sec. 4.3)
__device__ inline void wm_chunk_offsets(OffShared& sh, uint32_t b, uint32_t tau, uint32_t n, uint32_t* G0,
                                        uint64_t* const* words, bool natural = false)
{
    const uint32_t ngroups = (2u << tau) - 1u;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    for (int j = (int)tau - 1; j >= 0; j--) {
        if (threadIdx.x < (1u << j)) {
            const uint32_t c = gidx(j + 1, 2 * threadIdx.x), g = gidx(j, threadIdx.x);
            sh.cj[g] = sh.cj[c] + sh.cj[c + 1];
            sh.tj[g] = sh.tj[c] + sh.tj[c + 1];
        }
        __syncthreads();
    }
    for (uint32_t j = wave; j <= tau; j += HT / 64) {
        const uint32_t nk = 1u << j;
        uint32_t run = 0;
        for (uint32_t r0 = 0; r0 < nk; r0 += 64) {
            const uint32_t r = r0 + lane;
            const uint32_t u = r < nk ? (natural ? r : brev(r, j)) : 0;
            const uint32_t v = r < nk ? sh.tj[gidx(j, u)] : 0;
            uint32_t t;
            const uint32_t ex = wave_excl_scan(v, &t);
            if (r < nk) sh.bs[gidx(j, u)] = run + ex;
            run += t;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < ngroups; i += HT) {
        const uint32_t g0 = sh.bs[i] + sh.cj[i];
        G0[(uint64_t)b * MAXG + i] = g0;
        const uint32_t j = 31 - __clz(i + 1);
        // a word that two chunks share is or-ed into; it must start at zero
        if (j < tau && (g0 & 63u) && g0 < n) words[j][g0 >> 6] = 0;
    }
    if (b == 0 && threadIdx.x < tau && (n & 63u)) words[threadIdx.x][(n - 1) >> 6] = 0;
}

struct OffArgs {
    const uint32_t* PH;      // [2^tau][K] exclusive prefix of the counts over chunks
    const uint32_t* totals;  // [2^tau]
    uint32_t* G0;
    uint64_t* words[8];
    uint32_t K, tau, n;
    uint32_t natural;        // runs in key order (a tree built in one pass)
};

__global__ void __launch_bounds__(HT)
wm_offsets_k(OffArgs a)
{
    __shared__ OffShared sh;
    const uint32_t b = blockIdx.x, tau = a.tau;
    if (threadIdx.x < (1u << tau)) {
        sh.cj[gidx(tau, threadIdx.x)] = a.PH[(uint64_t)threadIdx.x * a.K + b];
        sh.tj[gidx(tau, threadIdx.x)] = a.totals[threadIdx.x];
    }
    wm_chunk_offsets(sh, b, tau, a.n, a.G0, a.words, a.natural != 0);
}


}  // namespace
