// wv_scan.hip -- device-wide exclusive prefix sum (the prefix-sum primitive
// of Sec. 2: returns (0, X0, X0+X1, ...) and the overall sum).
//
// Reduce-then-scan over tiles of 2048 items: per-tile sums, one block scans
// the tile sums, then every tile rescans its items with its base (one
// workgroup per column does it all when a column fits one tile).  Several
// independent columns can be scanned at once: item i of column c is
// in[i * ncols + c].
#include "wv_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// exclusive scan of one value per thread across the block; returns the
// exclusive prefix, *total gets the block sum
__device__ inline uint64_t block_excl_scan(uint64_t v, uint64_t* total)
{
    __shared__ uint64_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc = wv_wave_incl_scan64(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (int w = 0; w < SCAN_THREADS / 64; w++) {
        if (w < wave) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__global__ void __launch_bounds__(SCAN_THREADS)
scan_reduce_k(const uint32_t* __restrict__ in, uint64_t count, uint32_t ncols, uint64_t* __restrict__ partial)
{
    const uint32_t col = blockIdx.y;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        uint64_t i = base + (uint64_t)k * SCAN_THREADS + threadIdx.x;
        if (i < count) s += in[i * ncols + col];
    }
    uint64_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partial[(uint64_t)col * gridDim.x + blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS)
scan_top_k(uint64_t* __restrict__ partial, uint64_t nparts, uint64_t* __restrict__ totals)
{
    const uint32_t col = blockIdx.x;
    uint64_t* p = partial + (uint64_t)col * nparts;
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nparts; base += SCAN_THREADS) {
        uint64_t i = base + threadIdx.x;
        uint64_t v = i < nparts ? p[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan(v, &tot);
        if (i < nparts) p[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[col] = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS)
scan_down_k(const uint32_t* __restrict__ in, uint64_t count, uint32_t ncols,
            const uint64_t* __restrict__ partial, uint64_t* __restrict__ out)
{
    const uint32_t col = blockIdx.y;
    const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        uint64_t i = base + k;
        v[k] = i < count ? in[i * ncols + col] : 0u;
        s += v[k];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(s, &tot) + partial[(uint64_t)col * gridDim.x + blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; k++) {
        uint64_t i = base + k;
        if (i < count) out[i * ncols + col] = ex;
        ex += v[k];
    }
}

// the whole scan of one column in one workgroup, when it fits one tile
__global__ void __launch_bounds__(SCAN_THREADS)
scan_one_k(const uint32_t* __restrict__ in, uint64_t count, uint32_t ncols, uint64_t* __restrict__ out,
           uint64_t* __restrict__ totals)
{
    const uint32_t col = blockIdx.x;
    const uint64_t base = (uint64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint64_t s = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const uint64_t i = base + k;
        v[k] = i < count ? in[i * ncols + col] : 0u;
        s += v[k];
    }
    uint64_t tot;
    uint64_t ex = block_excl_scan(s, &tot);
    for (int k = 0; k < SCAN_ITEMS; k++) {
        const uint64_t i = base + k;
        if (i < count) out[i * ncols + col] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) totals[col] = tot;
}

}  // namespace

uint64_t wv_scan_partials(uint64_t count, uint32_t ncols)
{
    uint64_t parts = wv_cdiv(count ? count : 1, SCAN_TILE);
    return parts * ncols;
}

hipError_t wv_scan_u32(const uint32_t* in, uint64_t* out, uint64_t count, uint32_t ncols,
                       uint64_t* partial, uint64_t* totals, hipStream_t s)
{
    const uint64_t parts = wv_cdiv(count ? count : 1, SCAN_TILE);
    if (parts == 1) {   // one tile per column: one launch
        scan_one_k<<<ncols, SCAN_THREADS, 0, s>>>(in, count, ncols, out, totals);
        return hipGetLastError();
    }
    dim3 grid((uint32_t)parts, ncols);
    // count == 0 still runs one reduce block per column, which writes 0
    scan_reduce_k<<<grid, SCAN_THREADS, 0, s>>>(in, count, ncols, partial);
    scan_top_k<<<ncols, SCAN_THREADS, 0, s>>>(partial, parts, totals);
    if (count) scan_down_k<<<grid, SCAN_THREADS, 0, s>>>(in, count, ncols, partial, out);
    return hipGetLastError();
}
