// Scan and stable LSD radix sort for gfx950 (wave64).
//
// Scan: three phases (tile sums, one-block scan of the tile sums, tile
// scan + offset), deterministic.  Radix sort: 8-bit digits; per pass an
// up-sweep histogram per 2048-key tile (LDS atomics), a digit-major scan of
// the histograms, and a down-sweep that ranks keys stably inside the tile
// with wave64 ballots (match-by-digit from 8 ballots, popcount of the lower
// lanes) and per-wave digit counts in LDS.
#include "dem_internal.h"

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

constexpr int RADIX_THREADS = 256;
constexpr int RADIX_ITEMS = 8;
constexpr int RADIX_TILE = RADIX_THREADS * RADIX_ITEMS;
constexpr int RADIX_WAVES = RADIX_THREADS / 64;

__device__ inline uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(x, d, 64);
        if (lane >= d) x += t;
    }
    return x;
}

// Exclusive scan over a 256-thread block; returns the block total in *total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; ++k) {
        uint32_t s = wsum[k];
        off += (k < wid) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return inc - v + off;
}

__global__ void __launch_bounds__(256) k_fill(uint32_t *p, int64_t n, uint32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void __launch_bounds__(256) k_copy(uint32_t *d, const uint32_t *s, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = s[i];
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t *in, int64_t n,
                                                              uint32_t *partials)
{
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + (int64_t)k * SCAN_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Tile scan + offset.  Each block adds up the sums of the tiles before it
// (strided over its threads, then a block reduction; integer sums are exact
// in any order), so no separate pass over the tile sums is needed.  Also
// writes out[n] = total, an optional copy of the result, and an optional
// capacity check of the total.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const uint32_t *in, uint32_t *out,
                                                            uint32_t *out2, int64_t n,
                                                            const uint32_t *partials, int64_t nb,
                                                            DevCounters *ctr, int64_t cap, int buf)
{
    __shared__ uint32_t red[SCAN_THREADS / 64];
    uint32_t pre = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_THREADS) pre += partials[b];
    for (int d = 32; d > 0; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
    __syncthreads();
    pre = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; ++k) pre += red[k];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, &tot) + pre;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = base + k;
        if (i < n) {
            out[i] = ex;
            if (out2) out2[i] = ex;
        }
        ex += v[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == SCAN_THREADS - 1) {
        // ex is now the grand total (last thread of the last tile)
        out[n] = ex;
        if (out2) out2[n] = ex;
        if (ctr) {
            ctr->n_contacts[buf] = ex;
            if ((int64_t)ex > cap) {
                ctr->overflow[buf] = 1u;
                atomicMax(&ctr->required, ex);
            } else {
                ctr->overflow[buf] = 0u;
            }
        }
    }
}

__global__ void __launch_bounds__(RADIX_THREADS) k_radix_up(const uint32_t *keys, int64_t n, int shift,
                                                           uint32_t *hist, int64_t nblk)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
#pragma unroll
    for (int k = 0; k < RADIX_ITEMS; ++k) {
        int64_t i = base + (int64_t)k * RADIX_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(RADIX_THREADS) k_radix_down(const uint32_t *keys, const uint32_t *vals,
                                                             uint32_t *keys_out, uint32_t *vals_out,
                                                             int64_t n, int shift,
                                                             const uint32_t *offsets, int64_t nblk)
{
    __shared__ uint32_t running[256];
    __shared__ uint32_t wcnt[RADIX_WAVES][256];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    running[tid] = offsets[(int64_t)tid * nblk + blockIdx.x];
#pragma unroll
    for (int w = 0; w < RADIX_WAVES; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    for (int k = 0; k < RADIX_ITEMS; ++k) {
        int64_t i = base + (int64_t)k * RADIX_THREADS + tid;
        bool valid = i < n;
        uint32_t key = valid ? keys[i] : 0u;
        uint32_t val = valid ? vals[i] : 0u;
        uint32_t d = (key >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot((d >> b) & 1u);
            match &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(match & lt);
        if (valid && rank == 0) wcnt[wid][d] = (uint32_t)__popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t pos = running[d] + rank;
            for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < RADIX_WAVES; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        running[tid] += add;
        __syncthreads();
    }
}

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 1 << 16)
{
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

int64_t scan_tmp_elems(int64_t n)
{
    return (n + SCAN_TILE - 1) / SCAN_TILE + 2;
}

int64_t radix_hist_elems(int64_t n)
{
    return 256 * ((n + RADIX_TILE - 1) / RADIX_TILE + 1) + 1;
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, value);
}

void launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, dst, src, n);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                        hipStream_t s, uint32_t *out2, DevCounters *ctr, int64_t cap, int buf)
{
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) {
        launch_fill_u32(out, 1, 0u, s);
        if (out2) launch_fill_u32(out2, 1, 0u, s);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, out, out2, n,
                       partials, nb, ctr, cap, buf);
}

void radix_sort_u32(uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt,
                    int64_t n, int bits, uint32_t *hist, uint32_t *partials, hipStream_t s)
{
    if (n <= 1) return;
    int64_t nblk = (n + RADIX_TILE - 1) / RADIX_TILE;
    int passes = (bits + 7) / 8;
    uint32_t *ki = *keys, *vi = *vals, *ko = *keys_alt, *vo = *vals_alt;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_up, dim3((unsigned)nblk), dim3(RADIX_THREADS), 0, s, ki, n, shift,
                           hist, nblk);
        scan_exclusive_u32(hist, hist, 256 * nblk, partials, s);
        hipLaunchKernelGGL(k_radix_down, dim3((unsigned)nblk), dim3(RADIX_THREADS), 0, s, ki, vi, ko,
                           vo, n, shift, hist, nblk);
        uint32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    // after an odd number of passes the result sits in the alt buffers: swap roles
    *keys = ki;
    *vals = vi;
    *keys_alt = ko;
    *vals_alt = vo;
}
