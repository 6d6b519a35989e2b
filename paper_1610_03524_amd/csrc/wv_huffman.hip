// wv_huffman.hip -- canonical Huffman codewords computed on the device.
//
// The codewords shape a Huffman-shaped tree (Sec. 4.3, "Arbitrarily-shaped
// binary trees"); the paper notes they can be generated in parallel in
// O(sigma + log n) depth.  One workgroup does it for up to
// WT_HUFFMAN_DEV_MAX_SIGMA symbols, all in LDS, with the rule of
// wt_huffman_codes: leaves of nonzero count ordered by (count, symbol), a
// two-queue merge (merged nodes in creation order, the leaf taken on equal
// weight), lengths = leaf depths, one coded symbol gets length 1, codes
// assigned in (length, symbol) order.
//   1. keys (count, symbol) of the present symbols, bitonic sort;
//   2. the merge, sequential by construction (O(sigma) depth), by one thread;
//   3. every leaf walks up to the root for its depth (parallel);
//   4. keys (length, symbol), bitonic sort; a leaf's code is the first code
//      of its length plus its rank among that length's symbols.
#include "wv_internal.h"

namespace {

constexpr uint32_t HF_T = 1024;
constexpr uint32_t HF_MAX = WT_HUFFMAN_DEV_MAX_SIGMA;   // leaves
constexpr uint32_t HF_SYM_BITS = 13;                    // symbol bits of a sort key (HF_MAX <= 2^13)
constexpr uint32_t HF_NONE = 0xFFFFu;

// ascending bitonic sort of a[0..P) (P a power of two) by the whole workgroup
__device__ void bitonic(uint64_t* a, uint32_t P)
{
    for (uint32_t k = 2; k <= P; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < P; i += HF_T) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint64_t x = a[i], y = a[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
        }
    __syncthreads();
}

__global__ void __launch_bounds__(HF_T)
huffman_k(const uint64_t* __restrict__ counts, uint32_t sigma, uint64_t* __restrict__ codes,
          uint32_t* __restrict__ lens, int32_t* __restrict__ status)
{
    __shared__ uint64_t key[HF_MAX];        // (count, symbol), later (length, symbol)
    __shared__ uint64_t mw[HF_MAX];         // weights of merged nodes, in creation order
    __shared__ uint16_t up[2 * HF_MAX];     // parent of every node (leaves first)
    __shared__ uint32_t nleaf, bad;
    __shared__ uint32_t lcount[34], first_code[34], start[34];
    const uint32_t tid = threadIdx.x;
    uint32_t P = 1;
    while (P < sigma) P <<= 1;
    if (tid == 0) { nleaf = 0; bad = 0; }
    if (tid < 34) lcount[tid] = 0;
    for (uint32_t x = tid; x < sigma; x += HF_T) { codes[x] = 0; lens[x] = 0; }
    __syncthreads();
    for (uint32_t x = tid; x < P; x += HF_T) {
        const uint64_t c = x < sigma ? counts[x] : 0;
        key[x] = c ? ((c << HF_SYM_BITS) | x) : ~0ull;
        if (c) atomicAdd(&nleaf, 1u);
    }
    bitonic(key, P);
    const uint32_t k = nleaf;
    if (k == 1 && tid == 0) lens[key[0] & ((1u << HF_SYM_BITS) - 1)] = 1;
    if (k <= 1) {
        if (tid == 0) *status = WT_OK;
        return;
    }
    // 2. the merge (nodes 0..k-1: leaves in sorted order, k..2k-2: merged)
    if (tid == 0) {
        uint32_t lf = 0, mf = 0, made = 0;
        while (made < k - 1) {
            uint32_t pick[2];
            uint64_t w = 0;
            for (int t = 0; t < 2; t++) {
                const bool leaf_ok = lf < k, merged_ok = mf < made;
                const uint64_t lw = leaf_ok ? (key[lf] >> HF_SYM_BITS) : 0;
                if (leaf_ok && (!merged_ok || lw <= mw[mf])) {
                    w += lw;
                    pick[t] = lf++;
                } else {
                    w += mw[mf];
                    pick[t] = k + mf++;
                }
            }
            up[pick[0]] = up[pick[1]] = (uint16_t)(k + made);
            mw[made++] = w;
        }
        up[2 * k - 2] = HF_NONE;   // the root
    }
    __syncthreads();
    // 3. depths: every leaf walks up (a length over 32 is refused)
    for (uint32_t t = tid; t < k; t += HF_T) {
        uint32_t d = 0, v = t;
        while (up[v] != HF_NONE && d <= 32) {
            v = up[v];
            d++;
        }
        if (d > 32) atomicOr(&bad, 1u);
        atomicAdd(&lcount[min(d, 33u)], 1u);
        // the sort key of step 4: (length, symbol)
        key[t] = ((uint64_t)d << HF_SYM_BITS) | (key[t] & ((1u << HF_SYM_BITS) - 1));
    }
    for (uint32_t t = k + tid; t < P; t += HF_T) key[t] = ~0ull;
    __syncthreads();
    if (bad) {
        if (tid == 0) *status = WT_EUNSUP;
        return;
    }
    // 4. canonical codes: the first code and first sorted position of every
    // length (codes of one length are consecutive, the next length starts at
    // (last + 1) << 1 per extra bit)
    if (tid == 0) {
        uint64_t c = 0;
        uint32_t s = 0, prev = 0;
        bool any = false;
        for (uint32_t l = 1; l <= 32; l++) {
            if (!lcount[l]) continue;
            if (any) c = (c + 1) << (l - prev);
            first_code[l] = (uint32_t)c;
            start[l] = s;
            c += lcount[l] - 1;   // the last code of this length
            s += lcount[l];
            prev = l;
            any = true;
        }
    }
    bitonic(key, P);
    for (uint32_t t = tid; t < k; t += HF_T) {
        const uint32_t l = (uint32_t)(key[t] >> HF_SYM_BITS);
        const uint32_t x = (uint32_t)(key[t] & ((1u << HF_SYM_BITS) - 1));
        lens[x] = l;
        codes[x] = (uint64_t)first_code[l] + (t - start[l]);
    }
    if (tid == 0) *status = WT_OK;
}

}  // namespace

extern "C" int wt_huffman_codes_dev(const uint64_t* counts, uint32_t sigma, uint64_t* codes, uint32_t* code_len,
                                    int32_t* status, void* stream)
{
    if (!counts || !codes || !code_len || !status || sigma == 0) return WT_EINVAL;
    if (sigma > WT_HUFFMAN_DEV_MAX_SIGMA) return WT_EUNSUP;
    huffman_k<<<1, HF_T, 0, (hipStream_t)stream>>>(counts, sigma, codes, code_len, status);
    return hipGetLastError() == hipSuccess ? WT_OK : WT_EHIP;
}
