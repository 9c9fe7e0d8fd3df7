// Scan and stable LSD radix sort for gfx950 (wave64).
//
// Scan: tile sums, then tile scan + offset, deterministic.  A tile is 1024
// values, four per thread loaded and stored as one 16-byte vector (a wave
// touches 1 KiB contiguously).  With few tiles each block adds up the tile
// sums before it itself; with many, a one-block pass scans the tile sums
// in between.  Radix sort: 8-bit digits; per pass an
// up-sweep histogram per 2048-key tile (LDS atomics), a digit-major scan of
// the histograms, and a down-sweep that ranks keys stably inside the tile
// with wave64 ballots (match-by-digit from 8 ballots, popcount of the lower
// lanes) and per-wave digit counts in LDS.
#include "dem_internal.h"

#include <algorithm>

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
constexpr int64_t SCAN_DIRECT_TILES = 2048;   // up to this many tiles: no separate pass over tile sums
constexpr int SPINE_THREADS = 1024;

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

// Zero-fills up to three arrays in one launch (blockIdx.y picks the array).
__global__ void __launch_bounds__(256) k_zero3(uint32_t *p0, int64_t n0, uint32_t *p1, int64_t n1, uint32_t *p2,
                                               int64_t n2)
{
    uint32_t *p = blockIdx.y == 0 ? p0 : (blockIdx.y == 1 ? p1 : p2);
    const int64_t n = blockIdx.y == 0 ? n0 : (blockIdx.y == 1 ? n1 : n2);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

__global__ void __launch_bounds__(256) k_copy(uint32_t *d, const uint32_t *s, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) d[i] = s[i];
}

// Loads the four values at i..i+3 (i a multiple of 4, the array 16-byte
// aligned); values at or past n read as 0.
__device__ inline uint4 load4(const uint32_t *in, int64_t i, int64_t n)
{
    if (i + 3 < n) return *reinterpret_cast<const uint4 *>(in + i);
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i < n) v.x = in[i];
    if (i + 1 < n) v.y = in[i + 1];
    if (i + 2 < n) v.z = in[i + 2];
    return v;
}

__device__ inline void store4(uint32_t *out, int64_t i, int64_t n, uint4 v)
{
    if (i + 3 < n) {
        *reinterpret_cast<uint4 *>(out + i) = v;
        return;
    }
    if (i < n) out[i] = v.x;
    if (i + 1 < n) out[i + 1] = v.y;
    if (i + 2 < n) out[i + 2] = v.z;
}

// One scan of a launch; a launch scans one or two arrays of the same
// length (blockIdx.y picks the job).
struct ScanJob {
    const uint32_t *in;
    uint32_t *out, *out2;    // out2: optional copy of the result
    uint32_t *partials;      // tile sums of this job
    DevCounters *ctr;        // optional capacity check of the total
    int64_t cap;
    int buf;
};

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(ScanJob j0, ScanJob j1, int64_t n)
{
    const ScanJob &j = blockIdx.y == 0 ? j0 : j1;
    const uint4 v = load4(j.in, (int64_t)blockIdx.x * SCAN_TILE + 4 * (int64_t)threadIdx.x, n);
    uint32_t tot;
    block_excl_scan((v.x + v.y) + (v.z + v.w), &tot);
    if (threadIdx.x == 0) j.partials[blockIdx.x] = tot;
}

// One block per job: partials[0..nb) <- their exclusive prefix sums.  The
// tile sums are taken in chunks of SPINE_THREADS * 4 consecutive values
// (thread t holds values 4t .. 4t + 3 of the chunk, so a wave's loads are
// contiguous): a block scan of each chunk plus the carry of the chunks
// before it.
__global__ void __launch_bounds__(SPINE_THREADS) k_scan_spine(ScanJob j0, ScanJob j1, int64_t nb)
{
    __shared__ uint32_t wsum[SPINE_THREADS / 64];
    uint32_t *partials = blockIdx.y == 0 ? j0.partials : j1.partials;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int64_t CHUNK = (int64_t)SPINE_THREADS * 4;
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += CHUNK) {
        const int64_t i0 = c0 + 4 * (int64_t)threadIdx.x;
        uint32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k < nb ? partials[i0 + k] : 0u;
        const uint32_t s = (v[0] + v[1]) + (v[2] + v[3]);
        uint32_t inc = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        uint32_t off = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < SPINE_THREADS / 64; ++k) {
            const uint32_t w = wsum[k];
            off += k < wid ? w : 0u;
            tot += w;
        }
        uint32_t run = carry + off + (inc - s);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < nb) partials[i0 + k] = run;
            run += v[k];
        }
        carry += tot;
        __syncthreads();   // (wsum is rewritten by the next chunk)
    }
}

// Tile scan + offset.  The tile is loaded first; its offset is either the
// sum of the tile sums before it (few tiles: strided over the threads, then
// a block reduction; integer sums are exact in any order) or, after the
// spine pass, partials[blockIdx.x].  Also writes out[n] = total, the
// optional copy, and the optional capacity check of the total.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(ScanJob j0, ScanJob j1, int64_t n, int64_t nb,
                                                            int spine)
{
    __shared__ uint32_t red[SCAN_THREADS / 64];
    const ScanJob &j = blockIdx.y == 0 ? j0 : j1;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + 4 * (int64_t)threadIdx.x;
    const uint4 v = load4(j.in, base, n);
    uint32_t pre = 0;
    if (spine) {
        pre = j.partials[blockIdx.x];
    } else {
        for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_THREADS) pre += j.partials[b];
        for (int d = 32; d > 0; d >>= 1) pre += __shfl_xor(pre, d, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
        __syncthreads();
        pre = 0;
#pragma unroll
        for (int k = 0; k < SCAN_THREADS / 64; ++k) pre += red[k];
    }
    const uint32_t s = (v.x + v.y) + (v.z + v.w);
    uint32_t tot;
    const uint32_t ex = block_excl_scan(s, &tot) + pre;
    uint4 o;
    o.x = ex;
    o.y = o.x + v.x;
    o.z = o.y + v.y;
    o.w = o.z + v.z;
    store4(j.out, base, n, o);
    if (j.out2) store4(j.out2, base, n, o);
    if (blockIdx.x == nb - 1 && threadIdx.x == SCAN_THREADS - 1) {
        // the last thread of the last tile (values past n read as 0)
        const uint32_t total = ex + s;
        j.out[n] = total;
        if (j.out2) j.out2[n] = total;
        if (j.ctr) {
            j.ctr->n_contacts[j.buf] = total;
            if ((int64_t)total > j.cap) {
                j.ctr->overflow[j.buf] = 1u;
                atomicMax(&j.ctr->required, total);
            } else {
                j.ctr->overflow[j.buf] = 0u;
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

void launch_zero3(uint32_t *p0, int64_t n0, uint32_t *p1, int64_t n1, uint32_t *p2, int64_t n2, hipStream_t s)
{
    const int64_t m = std::max(n0, std::max(n1, n2));
    if (m <= 0) return;
    hipLaunchKernelGGL(k_zero3, dim3(grid_for(m, 256, 4096), 3), dim3(256), 0, s, p0, p0 ? n0 : 0, p1,
                       p1 ? n1 : 0, p2, p2 ? n2 : 0);
}

void launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, dst, src, n);
}

static void scan_jobs(const ScanJob &j0, const ScanJob &j1, int njobs, int64_t n, hipStream_t s)
{
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) {
        launch_fill_u32(j0.out, 1, 0u, s);
        if (j0.out2) launch_fill_u32(j0.out2, 1, 0u, s);
        if (njobs > 1) {
            launch_fill_u32(j1.out, 1, 0u, s);
            if (j1.out2) launch_fill_u32(j1.out2, 1, 0u, s);
        }
        return;
    }
    const dim3 grid((unsigned)nb, (unsigned)njobs);
    hipLaunchKernelGGL(k_scan_reduce, grid, dim3(SCAN_THREADS), 0, s, j0, j1, n);
    const int spine = nb > SCAN_DIRECT_TILES ? 1 : 0;
    if (spine) hipLaunchKernelGGL(k_scan_spine, dim3(1, (unsigned)njobs), dim3(SPINE_THREADS), 0, s, j0, j1, nb);
    hipLaunchKernelGGL(k_scan_down, grid, dim3(SCAN_THREADS), 0, s, j0, j1, n, nb, spine);
}

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                        hipStream_t s, uint32_t *out2, DevCounters *ctr, int64_t cap, int buf)
{
    ScanJob j{in, out, out2, partials, ctr, cap, buf};
    scan_jobs(j, j, 1, n, s);
}

void scan_exclusive_u32_pair(const uint32_t *in0, uint32_t *out0, uint32_t *out0b, DevCounters *ctr, int64_t cap,
                             int buf, const uint32_t *in1, uint32_t *out1, uint32_t *out1b, int64_t n,
                             uint32_t *partials, hipStream_t s)
{
    ScanJob j0{in0, out0, out0b, partials, ctr, cap, buf};
    ScanJob j1{in1, out1, out1b, partials + scan_tmp_elems(n), nullptr, 0, 0};
    scan_jobs(j0, j1, 2, n, s);
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
