// Scan and stable LSD radix sort for gfx950 (wave64).
//
// Scan, deterministic (integer sums): with few tiles of 1024 values (four
// per thread loaded and stored as one 16-byte vector, so a wave touches
// 1 KiB contiguously), tile sums, then a tile scan where each block adds up
// the tile sums before it.  With many, one pass over tiles of 16384 values
// with decoupled look-back (Merrill and Garland's single-pass scan): each
// block takes its tile from a ticket counter, so every tile before it
// belongs to a block that has already started, publishes its tile sum,
// adds up the published sums and prefixes of the tiles before it, and
// publishes its own prefix.  Radix sort: 8-bit digits; per pass an
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
// single-pass scan: tiles of LB_SUB sub-tiles of SCAN_TILE values
constexpr int LB_SUB = 16;
constexpr int64_t LB_TILE = (int64_t)LB_SUB * SCAN_TILE;

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

// The total of a job: out[n], its copy, and the optional capacity check.
__device__ inline void scan_total(const ScanJob &j, int64_t n, uint32_t total)
{
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

// Tile scan + offset (few tiles).  The tile is loaded first; its offset is
// the sum of the tile sums before it (strided over the threads, then a
// block reduction; integer sums are exact in any order).  Also writes
// out[n] = total, the optional copy, and the optional capacity check of
// the total.
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(ScanJob j0, ScanJob j1, int64_t n, int64_t nb)
{
    __shared__ uint32_t red[SCAN_THREADS / 64];
    const ScanJob &j = blockIdx.y == 0 ? j0 : j1;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + 4 * (int64_t)threadIdx.x;
    const uint4 v = load4(j.in, base, n);
    uint32_t pre = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += SCAN_THREADS) pre += j.partials[b];
    for (int d = 32; d > 0; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
    __syncthreads();
    pre = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; ++k) pre += red[k];
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
    // the last thread of the last tile (values past n read as 0)
    if (blockIdx.x == nb - 1 && threadIdx.x == SCAN_THREADS - 1) scan_total(j, n, ex + s);
}

// Single-pass scan state in a job's partials: word 0 the ticket counter,
// then (from the next 8-byte boundary) one status word per tile: the flag
// in the high half (0 nothing yet, LB_AGG the tile's own sum, LB_PREFIX the
// sum of every value up to the tile's end), the sum in the low half.  The
// flag and the sum travel in one 64-bit word, so a reader that sees the
// flag sees its sum.
constexpr unsigned long long LB_AGG = 1ull << 32;
constexpr unsigned long long LB_PREFIX = 2ull << 32;

__device__ inline unsigned long long *lb_status(uint32_t *partials)
{
    return reinterpret_cast<unsigned long long *>(partials + 2 - (reinterpret_cast<uintptr_t>(partials) >> 2 & 1u));
}

// Clears the ticket and the tile statuses of each job before the pass.
__global__ void __launch_bounds__(256) k_scan_lb_init(ScanJob j0, ScanJob j1, int64_t nb)
{
    const ScanJob &j = blockIdx.y == 0 ? j0 : j1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) j.partials[0] = 0u;
    if (i < nb) lb_status(j.partials)[i] = 0ull;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_lookback(ScanJob j0, ScanJob j1, int64_t n, int64_t nb)
{
    __shared__ uint32_t wsum[LB_SUB][SCAN_THREADS / 64];
    __shared__ uint32_t s_tile, s_excl;
    const ScanJob &j = blockIdx.y == 0 ? j0 : j1;
    unsigned long long *st = lb_status(j.partials);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_tile = atomicAdd(&j.partials[0], 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * LB_TILE + 4 * (int64_t)threadIdx.x;
    // sub-tile k: thread t holds its values 4t .. 4t + 3
    uint4 v[LB_SUB];
    uint32_t sk[LB_SUB], inc[LB_SUB];
#pragma unroll
    for (int k = 0; k < LB_SUB; ++k) v[k] = load4(j.in, base + (int64_t)k * SCAN_TILE, n);
#pragma unroll
    for (int k = 0; k < LB_SUB; ++k) {
        sk[k] = (v[k].x + v[k].y) + (v[k].z + v[k].w);
        inc[k] = wave_incl_scan(sk[k]);
        if (lane == 63) wsum[k][wid] = inc[k];
    }
    __syncthreads();
    // per sub-tile: the offset of this wave and the sub-tile's sum
    uint32_t off[LB_SUB], agg = 0;
#pragma unroll
    for (int k = 0; k < LB_SUB; ++k) {
        uint32_t o = 0, t = 0;
#pragma unroll
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            const uint32_t x = wsum[k][w];
            o += w < wid ? x : 0u;
            t += x;
        }
        off[k] = agg + o;
        agg += t;
    }
    if (wid == 0) {
        // publish the tile's sum, then (tiles after the first) add up what
        // the tiles before it published, 64 at a time from the nearest one,
        // down to the nearest that holds a prefix
        if (lane == 0)
            __hip_atomic_store(&st[tile], (tile == 0 ? LB_PREFIX : LB_AGG) | agg, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint32_t excl = 0;
        if (tile > 0) {
            int64_t top = tile - 1;
            while (true) {
                const int64_t q = top - lane;
                const unsigned long long w =
                    q >= 0 ? __hip_atomic_load(&st[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_PREFIX;
                const unsigned long long fl = w & ~0xffffffffull;
                const uint64_t pm = __ballot(fl == LB_PREFIX);
                const uint64_t zm = __ballot(fl == 0ull);
                // lanes up to the nearest prefix are needed
                const int p = pm ? __builtin_ctzll(pm) : 64;
                const uint64_t need = p >= 63 ? ~0ull : ((1ull << (p + 1)) - 1ull);
                if (zm & need) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint32_t x = lane <= p ? (uint32_t)w : 0u;
                for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d, 64);
                excl += x;
                if (p < 64) break;
                top -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&st[tile], LB_PREFIX | (uint32_t)(excl + agg), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    const uint32_t excl = s_excl;
#pragma unroll
    for (int k = 0; k < LB_SUB; ++k) {
        uint4 o;
        o.x = excl + off[k] + (inc[k] - sk[k]);
        o.y = o.x + v[k].x;
        o.z = o.y + v[k].y;
        o.w = o.z + v[k].z;
        store4(j.out, base + (int64_t)k * SCAN_TILE, n, o);
        if (j.out2) store4(j.out2, base + (int64_t)k * SCAN_TILE, n, o);
    }
    // (values past n read as 0)
    if (tile == nb - 1 && threadIdx.x == 0) scan_total(j, n, excl + agg);
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
    // tile sums of the few-tile pass; the single-pass state (ticket, an
    // alignment word, two words per 16384-value tile) fits in the same room
    return (n + SCAN_TILE - 1) / SCAN_TILE + 8;
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
    if (nb <= SCAN_DIRECT_TILES) {
        const dim3 grid((unsigned)nb, (unsigned)njobs);
        hipLaunchKernelGGL(k_scan_reduce, grid, dim3(SCAN_THREADS), 0, s, j0, j1, n);
        hipLaunchKernelGGL(k_scan_down, grid, dim3(SCAN_THREADS), 0, s, j0, j1, n, nb);
        return;
    }
    const int64_t nl = (n + LB_TILE - 1) / LB_TILE;
    hipLaunchKernelGGL(k_scan_lb_init, dim3((unsigned)((nl + 255) / 256), (unsigned)njobs), dim3(256), 0, s, j0, j1,
                       nl);
    hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)nl, (unsigned)njobs), dim3(SCAN_THREADS), 0, s, j0, j1, n,
                       nl);
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
