// wv_wm_passes.hip -- the wavelet matrix built tau levels per pass.
//
// Sec. 4.3 ("Wavelet matrix") builds every tau-th level by an integer sort of
// the current sequence on the reversed tau bits below the levels already
// done, and the levels in between from the short tau-bit keys.  Here one pass
// handles tau consecutive levels l = a*tau + j (j = 0..tau-1):
//
//   * The sequence of the pass (S for the first pass, then the compacted
//     remaining key bits written by the previous pass) is cut into K
//     contiguous chunks, one workgroup each; a chunk is a sub-problem of the
//     domain decomposition of Sec. 4.2, processed tile after tile.
//   * Level a*tau + j holds bit j of the tau-bit digit in the order of a
//     stable sort by the first j digit bits, the most recent bit most
//     significant (the wavelet-matrix order).  Inside a tile that order is
//     produced by j stable 1-bit partitions in LDS; the tile's bits then form
//     2^j runs, one per key, each going to a contiguous range of the level at
//     an offset from the prefix sums of the per-chunk digit histograms
//     (the prefix-sum offsets of Sec. 4.1 / Sec. 4.2).
//   * Runs are written as 64-bit words.  A chunk carries the partial last
//     word of each run from tile to tile, so only the first and last word of
//     a chunk's run can be shared with another chunk; those "boundary" words
//     (Sec. 4.2) are zeroed beforehand and OR-ed atomically, every other word
//     is a plain store.
//   * After the last sub-level the remaining key bits are scattered to the
//     order of level (a+1)*tau (the next pass's input, the big-node sequence
//     of Sec. 3/4.1), compacted to the narrowest integer type.
//
// Kernels per pass: a histogram of the pass digit per chunk (the first pass
// also validates S), two small scans giving every chunk's run offsets and
// zeroing the boundary words, and the pass itself.  The rank directories and
// select samples of all levels follow (wv_directory.hip).
#include <algorithm>

#include "wv_wm_passes.h"
#include "wv_wm_core.h"

namespace {

// 8- and 16-bit keys in LDS: four workgroups per CU (8 waves per SIMD, 64
// VGPRs; byte keys need no scaling of their LDS index); 32-bit keys: LDS
// holds three workgroups per CU, so 6 waves per SIMD
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8)))
wm_pass8_k(PassArgs a)
{
    __shared__ PassShared<uint8_t> sh;
    wm_pass_chunk<uint8_t>(a, blockIdx.x, sh);
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8, 8)))
wm_pass16_k(PassArgs a)
{
    __shared__ PassShared<uint16_t> sh;
    wm_pass_chunk<uint16_t>(a, blockIdx.x, sh);
}

__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6, 6)))
wm_pass32_k(PassArgs a)
{
    __shared__ PassShared<uint32_t> sh;
    wm_pass_chunk<uint32_t>(a, blockIdx.x, sh);
}

template <typename IT>
__global__ void __launch_bounds__(HT)
wm_hist_k(const void* __restrict__ in, uint32_t n, uint32_t C, uint32_t K, uint32_t R, uint32_t tau,
          uint32_t keymask, uint32_t* __restrict__ H, uint32_t* __restrict__ status, uint32_t sigma)
{
    __shared__ uint32_t h[HWORDS];
    wm_hist_part<IT>(in, n, C, K, R, tau, keymask, H, status, sigma, blockIdx.x / HSPLIT, blockIdx.x % HSPLIT, h);
}

inline uint32_t width_bytes(uint32_t bits) { return bits <= 8 ? 1u : (bits <= 16 ? 2u : 4u); }

struct Geometry {
    uint32_t K, C;
};

// K chunks of C keys (a multiple of the tile): `blocks` chunks, else chunks
// of `tile` tiles, else one chunk per resident workgroup of the first pass
// (whose keys are the widest)
Geometry geometry(uint64_t n, uint32_t blocks, uint32_t tile, uint32_t L)
{
    const uint64_t tiles = wv_cdiv(n ? n : 1, T);
    uint64_t K = blocks ? blocks : (tile ? wv_cdiv(tiles, tile) : (L > 16 ? KRES32 : KRES16));
    K = std::min<uint64_t>(K, tiles);
    // a chunk length must fit 32 bits: at least two chunks near n = 2^32
    K = std::max<uint64_t>(K, wv_cdiv(n ? n : 1, 0x100000000ull - T));
    const uint64_t C = wv_cdiv(wv_cdiv(n ? n : 1, K), T) * T;
    return Geometry{(uint32_t)wv_cdiv(n ? n : 1, C), (uint32_t)C};
}

void launch_pass(const PassArgs& a, hipStream_t s)
{
    if (a.R <= 8) wm_pass8_k<<<a.K, NT, 0, s>>>(a);
    else if (a.R <= 16) wm_pass16_k<<<a.K, NT, 0, s>>>(a);
    else wm_pass32_k<<<a.K, NT, 0, s>>>(a);
}

__global__ void zero_u32_k(uint32_t* p, uint32_t count)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0;
}

void launch_hist(uint32_t in_bytes, const void* in, uint32_t n, const Geometry& geo, uint32_t R, uint32_t tau,
                 uint32_t keymask, uint32_t* H, uint32_t* status, uint32_t sigma, hipStream_t s)
{
    const uint32_t cells = (1u << tau) * geo.K;
    zero_u32_k<<<(cells + 255) / 256, 256, 0, s>>>(H, cells);
    const uint32_t grid = geo.K * HSPLIT;
    if (in_bytes == 1) wm_hist_k<uint8_t><<<grid, HT, 0, s>>>(in, n, geo.C, geo.K, R, tau, keymask, H, status, sigma);
    else if (in_bytes == 2) wm_hist_k<uint16_t><<<grid, HT, 0, s>>>(in, n, geo.C, geo.K, R, tau, keymask, H, status, sigma);
    else wm_hist_k<uint32_t><<<grid, HT, 0, s>>>(in, n, geo.C, geo.K, R, tau, keymask, H, status, sigma);
}

}  // namespace

int wv_wm_make_plan(uint64_t n, uint32_t sigma, uint32_t sym_bytes, const wt_tuning* tune, wv_wm_plan& p)
{
    const uint32_t L = wv_key_bits(sigma);
    uint32_t tau = tune && tune->tau ? tune->tau : 0;
    if (tau > 8) return WT_EINVAL;
    if (!tau) {
        const uint32_t passes = (L + 7) / 8;
        tau = (L + passes - 1) / passes;
    }
    tau = std::min(tau, L);
    const Geometry geo = geometry(n, tune ? tune->blocks : 0, tune ? tune->tile : 0, L);
    p.enabled = true;
    p.tree_order = false;
    p.profile = tune && (tune->flags & WT_FLAG_PROFILE);
    p.tau = tau;
    p.L = L;
    p.sym_bytes = sym_bytes;
    p.K = geo.K;
    p.C = geo.C;
    p.n = n;
    p.sigma = sigma;
    // payload buffers: widest remaining key after the first pass
    const uint32_t rem = L > tau ? L - tau : 0;
    const uint64_t pay = rem ? (uint64_t)std::max<uint64_t>(n, 1) * width_bytes(rem) : 0;
    uint64_t off = 0;
    auto bump = [&](uint64_t bytes) { uint64_t at = off; off = wv_round256(off + bytes); return at; };
    p.off_H = bump((uint64_t)256 * geo.K * 4);
    p.off_tot = bump(256 * 4);
    p.off_G0 = bump((uint64_t)geo.K * MAXG * 4);
    p.off_pay[0] = bump(pay);
    p.off_pay[1] = bump(L > 2 * tau ? pay : 0);
    // directory scratch for all levels at once
    p.dir = wv_span_dir_sizes(n, L);
    p.off_dir = bump(p.dir.bytes);
    p.ws_bytes = off;
    return WT_OK;
}

hipError_t wv_wm_levels(const wv_wm_plan& p, const void* S, uint64_t* const* level_words, uint32_t* status,
                        uint8_t* ws, hipStream_t s)
{
    const uint32_t L = p.L, n = (uint32_t)p.n;
    uint32_t* H = (uint32_t*)(ws + p.off_H);
    uint32_t* tot = (uint32_t*)(ws + p.off_tot);
    uint32_t* G0 = (uint32_t*)(ws + p.off_G0);
    const Geometry geo{p.K, p.C};
    const void* in = S;
    uint32_t in_bytes = p.sym_bytes;
    uint32_t keymask = L >= 32 ? ~0u : ((1u << L) - 1u);
    int side = 0;
    if (n) {
        for (uint32_t l0 = 0; l0 < L; l0 += p.tau) {
            const uint32_t tau = std::min(p.tau, L - l0);
            const uint32_t R = L - l0;
            const uint32_t rem = R - tau;
            const bool pr = p.profile;
            WV_TIMED(pr, s, "wm_hist",
                     launch_hist(in_bytes, in, n, geo, R, tau, keymask, H, l0 == 0 ? status : nullptr, p.sigma, s));
            WV_TIMED(pr, s, "wm_scan", (wm_scan_chunks_k<<<1u << tau, HT, 0, s>>>(H, geo.K, tot)));
            OffArgs oa{};
            oa.PH = H;
            oa.totals = tot;
            oa.G0 = G0;
            for (uint32_t j = 0; j < tau; j++) oa.words[j] = level_words[l0 + j];
            oa.K = geo.K;
            oa.tau = tau;
            oa.n = n;
            oa.natural = p.tree_order ? 1u : 0u;
            WV_TIMED(pr, s, "wm_offsets", (wm_offsets_k<<<geo.K, HT, 0, s>>>(oa)));
            PassArgs pa{};
            pa.in = in;
            pa.pay_out = rem ? (void*)(ws + p.off_pay[side]) : nullptr;
            for (uint32_t j = 0; j < tau; j++) pa.words[j] = oa.words[j];
            pa.G0 = G0;
            pa.n = n;
            pa.C = geo.C;
            pa.K = geo.K;
            pa.R = R;
            pa.tau = tau;
            pa.keymask = keymask;
            pa.in_bytes = in_bytes;
            pa.out_bytes = width_bytes(rem);
            WV_TIMED(pr, s, "wm_pass", launch_pass(pa, s));
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            in = pa.pay_out;
            in_bytes = width_bytes(rem);
            keymask = ~0u;
            side ^= 1;
        }
    }
    return hipSuccess;
}

hipError_t wv_wm_run(const wv_wm_plan& p, const void* S, uint8_t* image, const wv_layout_out& lay, uint8_t* ws,
                     const wv_dir_scratch&, hipStream_t s)
{
    uint64_t* words[WV_MAX_LEVELS];
    for (uint32_t l = 0; l < p.L; l++) words[l] = (uint64_t*)(image + lay.lv[l].bits_off);
    hipError_t e = wv_wm_levels(p, S, words, (uint32_t*)(image + 36), ws, s);
    if (e != hipSuccess) return e;
    return wv_span_directory(image, lay, 0, p.L, ws + p.off_dir, p.dir, s, p.profile);
}
