// Learned contact-detection interval for gfx950.
//
// Features: per feature cell (a cube of edge 8 (r_max + m) tiling the domain
// box from its low corner: four times the smallest bin edge), from the
// owners whose centre lies in it, relative to the state at the previous
// detection (the snapshot):
//   f1 log1p(|v_max - v_min| h K / m)     spread of velocities (relative speed)
//   f2 log1p(max|v - v_snap| K^2 h / (2 tau m))  acceleration since the snapshot
//   f3 sum of sphere volumes / cell volume (packing fraction)
//   f4 tau / K                              steps since the last detection
//   f5 log1p(max|v| h K / m)                absolute speed
//   f6 log1p(max|X - X_snap| / m)           margin consumed since the snapshot
// with K = DEM_MLP_KCAP steps, m the margin, h the step, tau the steps since the
// snapshot.  Per-cell maxima and minima use order-free integer atomics and
// the volume a fixed-point integer sum, so features are deterministic; the
// occupied cells are compacted in cell order with a scan.
//
// MLP 6-32-32-1 (tanh, tanh, linear), parameters W1[32x6] b1 W2[32x32] b2
// W3[1x32] b3.  Forward: one thread per sample, parameters in LDS.
// Backward (expectile loss): 64 samples per block keep activations and
// deltas in LDS; each thread then sums its parameters' gradient over the
// block's samples in sample order, writes a per-block partial, and a second
// kernel adds the partials in block order -- a fixed summation order.
#include "dem_device.h"
#include "../../include/dem.h"

#include <mutex>
#include <string>

namespace {

constexpr int H = 32;
constexpr int NF = DEM_MLP_NFEAT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * NF, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;
static_assert(NPARAM == DEM_MLP_NPARAM, "parameter count");
constexpr int BWD_SAMPLES = 64;
constexpr int RAW = 16;   // u32 words of raw accumulators per cell

inline unsigned nblocks(int64_t n, int t)
{
    int64_t g = (n + t - 1) / t;
    return (unsigned)(g < 1 ? 1 : g);
}

__device__ inline void load_params(const float *p, float *sp)
{
    for (int k = threadIdx.x; k < NPARAM; k += blockDim.x) sp[k] = p[k];
    __syncthreads();
}

__device__ inline float mlp_eval(const float *P, const float *x, float *h1, float *h2)
{
#pragma unroll 4
    for (int u = 0; u < H; ++u) {
        float s = P[OFF_B1 + u];
#pragma unroll
        for (int k = 0; k < NF; ++k) s += P[OFF_W1 + u * NF + k] * x[k];
        h1[u] = tanhf(s);
    }
#pragma unroll 4
    for (int u = 0; u < H; ++u) {
        float s = P[OFF_B2 + u];
        for (int k = 0; k < H; ++k) s += P[OFF_W2 + u * H + k] * h1[k];
        h2[u] = tanhf(s);
    }
    float y = P[OFF_B3];
    for (int k = 0; k < H; ++k) y += P[OFF_W3 + k] * h2[k];
    return y;
}

__global__ void __launch_bounds__(256) k_mlp_forward(const float *params, const float *X, float *Y, int64_t n)
{
    __shared__ float sp[NPARAM];
    load_params(params, sp);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[NF], h1[H], h2[H];
    for (int k = 0; k < NF; ++k) x[k] = X[i * NF + k];
    Y[i] = mlp_eval(sp, x, h1, h2);
}

__global__ void __launch_bounds__(BWD_SAMPLES) k_mlp_backward_block(const float *params, const float *X,
                                                                   const float *T, int64_t n, float tau,
                                                                   float *partial, float *loss_partial)
{
    __shared__ float sp[NPARAM];
    __shared__ float sx[BWD_SAMPLES][NF];
    __shared__ float sh1[BWD_SAMPLES][H + 1];
    __shared__ float sh2[BWD_SAMPLES][H + 1];
    __shared__ float sd1[BWD_SAMPLES][H + 1];
    __shared__ float sd2[BWD_SAMPLES][H + 1];
    __shared__ float sg[BWD_SAMPLES];
    __shared__ float sl[BWD_SAMPLES];
    load_params(params, sp);
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * BWD_SAMPLES + t;
    const float inv_n = 1.0f / (float)n;
    if (i < n) {
        float x[NF], h1[H], h2[H];
        for (int k = 0; k < NF; ++k) x[k] = X[i * NF + k];
        float y = mlp_eval(sp, x, h1, h2);
        float r = y - T[i];
        float w = r > 0.0f ? (1.0f - tau) : tau;
        float g = 2.0f * w * r * inv_n;
        sl[t] = w * r * r * inv_n;
        sg[t] = g;
        for (int k = 0; k < NF; ++k) sx[t][k] = x[k];
        for (int u = 0; u < H; ++u) {
            sh1[t][u] = h1[u];
            sh2[t][u] = h2[u];
            sd2[t][u] = g * sp[OFF_W3 + u] * (1.0f - h2[u] * h2[u]);
        }
        for (int k = 0; k < H; ++k) {
            float s = 0.0f;
            for (int u = 0; u < H; ++u) s += sp[OFF_W2 + u * H + k] * sd2[t][u];
            sd1[t][k] = s * (1.0f - h1[k] * h1[k]);
        }
    } else {
        sl[t] = 0.0f;
        sg[t] = 0.0f;
        for (int k = 0; k < NF; ++k) sx[t][k] = 0.0f;
        for (int u = 0; u < H; ++u) {
            sh1[t][u] = 0.0f;
            sh2[t][u] = 0.0f;
            sd2[t][u] = 0.0f;
            sd1[t][u] = 0.0f;
        }
    }
    __syncthreads();
    float *out = partial + (int64_t)blockIdx.x * NPARAM;
    for (int p = t; p < NPARAM; p += BWD_SAMPLES) {
        float s = 0.0f;
        if (p < OFF_B1) {
            int u = p / NF, k = p % NF;
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sd1[q][u] * sx[q][k];
        } else if (p < OFF_W2) {
            int u = p - OFF_B1;
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sd1[q][u];
        } else if (p < OFF_B2) {
            int u = (p - OFF_W2) / H, k = (p - OFF_W2) % H;
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sd2[q][u] * sh1[q][k];
        } else if (p < OFF_W3) {
            int u = p - OFF_B2;
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sd2[q][u];
        } else if (p < OFF_B3) {
            int k = p - OFF_W3;
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sg[q] * sh2[q][k];
        } else {
            for (int q = 0; q < BWD_SAMPLES; ++q) s += sg[q];
        }
        out[p] = s;
    }
    if (t == 0) {
        float s = 0.0f;
        for (int q = 0; q < BWD_SAMPLES; ++q) s += sl[q];
        loss_partial[blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_mlp_backward_sum(const float *partial, const float *loss_partial,
                                                         int64_t nblk, float *grad, float *loss)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < NPARAM) {
        float s = 0.0f;
        for (int64_t b = 0; b < nblk; ++b) s += partial[b * NPARAM + p];
        grad[p] = s;
    } else if (p == NPARAM) {
        float s = 0.0f;
        for (int64_t b = 0; b < nblk; ++b) s += loss_partial[b];
        loss[0] = s;
    }
}

__global__ void __launch_bounds__(256) k_mlp_adam(float *params, const float *grad, float *m, float *v,
                                                 float lr, float b1, float b2, float eps, float c1, float c2)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float g = grad[p];
    float mm = b1 * m[p] + (1.0f - b1) * g;
    float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    float mh = mm / c1, vh = vv / c2;
    params[p] = params[p] - lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
__device__ inline uint32_t ord_enc(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float ord_dec(uint32_t u)
{
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ inline uint32_t fcell_of(const Grid &g, double x, double y, double z)
{
    double c[3] = {x, y, z};
    int n[3] = {g.nx, g.ny, g.nz};
    uint32_t id[3];
    for (int k = 0; k < 3; ++k) {
        double t = floor((c[k] - g.lo[k]) * g.inv_b);
        int v;
        if (!(t >= 0.0)) v = 0;
        else if (t > (double)(n[k] - 1)) v = n[k] - 1;
        else v = (int)t;
        id[k] = (uint32_t)v;
    }
    return (id[2] * (uint32_t)g.ny + id[1]) * (uint32_t)g.nx + id[0];
}

__global__ void __launch_bounds__(256) k_feat_clear(uint32_t *raw, int64_t ncell)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncell * (RAW / 4)) return;
    reinterpret_cast<uint4 *>(raw)[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Per-owner contributions to its feature cell.  Each block takes
// FEAT_OWNERS consecutive owners, each wave 64 consecutive ones at a time.
// Consecutive owners are mostly spatial neighbours, so the lanes of a wave
// fall into a few runs of equal cells: a segmented scan over the lanes
// (integer max and sums, order-free) combines each run, and the last lane
// of a run adds it to the block's table of cells in LDS (LDS atomics, open
// addressing on the low bits of the cell id, so that neighbouring cells take
// neighbouring slots).  When the block is done, its table goes to the global
// accumulators a few cells per wave instruction, one lane per accumulator
// word, so that an instruction's atomics fall on the consecutive words of
// consecutive cells (a few cache lines) rather than on 64 cells spread over
// the grid.  A cell that finds the table full goes straight to the global
// accumulators.
// With snap_out set, each owner's current position and velocity are
// written there after its snapshot is read (snap_out may equal snap: the
// thread that reads a record writes it).  With cellmap set, each owner's
// cell is written there (the training-log tools use it).
constexpr int FEAT_WAVE_ITERS = 8;
constexpr int64_t FEAT_OWNERS = 4 * 64 * FEAT_WAVE_ITERS;   // 2048
constexpr int FEAT_SLOTS = 512;
constexpr uint32_t FEAT_EMPTY = 0xffffffffu;
// Per cell (RAW words, zero when cleared), every word but the volume a
// maximum: words 0-2 the largest encoded velocity component, 3-5 the
// complement of the smallest (~enc: the complement turns the minimum into a
// maximum), 6-8 max dv, va, dx (non-negative float bits), 10-11 the volume
// (u64 sum).  The complement of an encoded value is zero only for one NaN
// pattern, so a cell is occupied once word 3 is non-zero.
constexpr int FEAT_MAXW = 9;

__device__ inline void feat_global_add(uint32_t *rw, const uint32_t *a, unsigned long long vol)
{
    for (int k = 0; k < FEAT_MAXW; ++k) atomicMax(&rw[k], a[k]);
    atomicAdd(reinterpret_cast<unsigned long long *>(&rw[10]), vol);
}

__global__ void __launch_bounds__(256) k_feat_accum(RecBuf rec, const SnapRec *snap, SnapRec *snap_out,
                                                   const float *ovol, Origin org, Grid fg, uint32_t *raw,
                                                   uint32_t *cellmap, int64_t No, bool nt)
{
    __shared__ uint32_t tkey[FEAT_SLOTS];
    __shared__ uint32_t tval[FEAT_SLOTS][FEAT_MAXW];
    __shared__ unsigned long long tvol[FEAT_SLOTS];
    __shared__ uint4 lrec[4][192];
    for (int k = threadIdx.x; k < FEAT_SLOTS; k += blockDim.x) {
        tkey[k] = FEAT_EMPTY;
        for (int j = 0; j < FEAT_MAXW; ++j) tval[k][j] = 0u;
        tvol[k] = 0ull;
    }
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63u);
    const int wv = (int)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < FEAT_WAVE_ITERS; ++it) {
        const int64_t ow = (int64_t)blockIdx.x * FEAT_OWNERS + (int64_t)(wv * FEAT_WAVE_ITERS + it) * 64;
        if (ow >= No) break;
        const int64_t o = ow + lane;
        const bool valid = o < No;
        const uint32_t nv = (uint32_t)(No - ow < 64 ? No - ow : 64);
        // the wave's records through LDS, in contiguous 1 KiB loads (of
        // hot parts only where records are split: the features need
        // position and velocity)
        rec_copy(rec_lds(lrec[wv], rec), 0, rec, ow, nv, lane, false);
        SnapRec sr{};
        float vo = 0.0f;
        if (valid) {
            sr = snap[o];
            vo = ovol[o];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t c = FEAT_EMPTY;
        uint32_t a[FEAT_MAXW] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        unsigned long long iv = 0ull;
        if (valid) {
            const OwnerRec r = load_rec_hot(rec_lds(lrec[wv], rec), lane);
            double X[3], Xs[3];
            for (int k = 0; k < 3; ++k) {
                X[k] = decode_axis(r.vox, r.off[k], org.o[k], k);
                Xs[k] = decode_axis(sr.vox, sr.off[k], org.o[k], k);
            }
            c = fcell_of(fg, X[0], X[1], X[2]);
            if (cellmap) cellmap[o] = c;
            for (int k = 0; k < 3; ++k) {
                const uint32_t e = ord_enc(r.v[k]);
                a[k] = e;
                a[3 + k] = ~e;
            }
            const float dv0 = r.v[0] - sr.v[0], dv1 = r.v[1] - sr.v[1], dv2 = r.v[2] - sr.v[2];
            const float dv = sqrtf((dv0 * dv0 + dv1 * dv1) + dv2 * dv2);
            const float va = sqrtf((r.v[0] * r.v[0] + r.v[1] * r.v[1]) + r.v[2] * r.v[2]);
            const double d0 = X[0] - Xs[0], d1 = X[1] - Xs[1], d2 = X[2] - Xs[2];
            const float dx = (float)sqrt((d0 * d0 + d1 * d1) + d2 * d2);
            a[6] = __float_as_uint(dv);
            a[7] = __float_as_uint(va);
            a[8] = __float_as_uint(dx);
            // fixed-point volume in units of 1e-18 m^3
            iv = (unsigned long long)((double)vo * 1e18 + 0.5);
            if (snap_out) {
                // (a snapshot holds what a record's hot part holds: voxel
                // word, offsets, velocity; split records write it from the
                // staged hot parts below, in whole lines)
                if (nt && !rec.cold) {
                    st_nt(rec_hot0(r), reinterpret_cast<uint4 *>(snap_out + o));
                    st_nt(rec_hot1(r), reinterpret_cast<uint4 *>(snap_out + o) + 1);
                } else if (!nt) {
                    SnapRec nw;
                    nw.vox = r.vox;
                    for (int k = 0; k < 3; ++k) {
                        nw.off[k] = r.off[k];
                        nw.v[k] = r.v[k];
                    }
                    snap_out[o] = nw;
                }
            }
        }
        if (snap_out && nt && rec.cold) {
            // the staged hot parts are the wave's new snapshot records
            uint4 *d = reinterpret_cast<uint4 *>(snap_out + ow);
            for (uint32_t k = (uint32_t)lane; k < 2u * nv; k += 64u) st_nt(lrec[wv][k], d + k);
        }
        // runs of equal cells over the lanes; the scan combines each run
        const uint32_t cprev = (uint32_t)__shfl_up((int)c, 1, 64);
        const bool head = lane == 0 || cprev != c;
        const uint64_t heads = __ballot(head);
        const int seg0 = 63 - __clzll((long long)(heads & (below | (1ull << lane))));
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const bool take = lane - d >= seg0;
            uint32_t t[FEAT_MAXW];
#pragma unroll
            for (int k = 0; k < FEAT_MAXW; ++k) t[k] = (uint32_t)__shfl_up((int)a[k], d, 64);
            const unsigned long long tv = (unsigned long long)__shfl_up((long long)iv, d, 64);
            if (take) {
#pragma unroll
                for (int k = 0; k < FEAT_MAXW; ++k) a[k] = max(a[k], t[k]);
                iv += tv;
            }
        }
        const uint32_t cnext = (uint32_t)__shfl_down((int)c, 1, 64);
        const bool tail = valid && (lane == 63 || cnext != c || !(o + 1 < No));
        if (tail) {
            uint32_t h = c & (FEAT_SLOTS - 1);
            int probe = 0;
            for (; probe < FEAT_SLOTS; ++probe) {
                const uint32_t old = atomicCAS(&tkey[h], FEAT_EMPTY, c);
                if (old == FEAT_EMPTY || old == c) break;
                h = (h + 1u) & (FEAT_SLOTS - 1);
            }
            if (probe < FEAT_SLOTS) {
                for (int k = 0; k < FEAT_MAXW; ++k) atomicMax(&tval[h][k], a[k]);
                atomicAdd(&tvol[h], iv);
            } else {
                feat_global_add(raw + (int64_t)c * RAW, a, iv);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();
    // the table out: RAW lanes per slot, lane w adding word w of its slot's
    // cell (the maxima, then the volume; the other words stay unused)
    static_assert(RAW == 16 && 256 % RAW == 0, "one lane per accumulator word");
    const int w = (int)(threadIdx.x & (RAW - 1));
    for (int k = (int)threadIdx.x / RAW; k < FEAT_SLOTS; k += 256 / RAW) {
        const uint32_t c = tkey[k];
        if (c == FEAT_EMPTY) continue;
        uint32_t *rw = raw + (int64_t)c * RAW;
        if (w < FEAT_MAXW) {
            const uint32_t v = tval[k][w];
            if (v != 0u) atomicMax(&rw[w], v);
        } else if (w == 10) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&rw[10]), tvol[k]);
        }
    }
}

__global__ void __launch_bounds__(256) k_feat_flags(const uint32_t *raw, int64_t ncell, uint32_t *flag)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    flag[c] = raw[c * RAW + 3] != 0u ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_feat_write(const uint32_t *raw, const uint32_t *pos, int64_t ncell,
                                                   float h, float margin, float tau, float K, float cell_vol,
                                                   float *out, uint32_t *cell_ids)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t *r = raw + c * RAW;
    if (r[3] == 0u) return;
    uint32_t p = pos[c];
    float vr[3];
    for (int k = 0; k < 3; ++k) vr[k] = ord_dec(r[k]) - ord_dec(~r[3 + k]);
    float spread = sqrtf((vr[0] * vr[0] + vr[1] * vr[1]) + vr[2] * vr[2]);
    float dv = __uint_as_float(r[6]), va = __uint_as_float(r[7]), dx = __uint_as_float(r[8]);
    unsigned long long iv = *reinterpret_cast<const unsigned long long *>(r + 10);
    float vol = (float)((double)iv * 1e-18);
    float t = tau < 1.0f ? 1.0f : tau;
    float *f = out + (int64_t)p * NF;
    f[0] = log1pf(spread * h * K / margin);
    f[1] = log1pf(dv * K * K * h / (2.0f * t * margin));
    f[2] = vol / cell_vol;
    f[3] = tau / K;
    f[4] = log1pf(va * h * K / margin);
    f[5] = log1pf(dx / margin);
    if (cell_ids) cell_ids[p] = (uint32_t)c;
}

// The features of every occupied cell straight into the network (the same
// arithmetic as k_feat_write and k_mlp_forward), the predicted remaining
// steps R = exp(y) - 1 of each (clamped at >= 0), and the minimum over the
// block's cells into slot[blockIdx.x] (3e38 when the block has none).
__device__ inline void feat_of_cell(const uint32_t *r, float h, float margin, float tau, float K, float cell_vol,
                                    float *f)
{
    float vr[3];
    for (int k = 0; k < 3; ++k) vr[k] = ord_dec(r[k]) - ord_dec(~r[3 + k]);
    const float spread = sqrtf((vr[0] * vr[0] + vr[1] * vr[1]) + vr[2] * vr[2]);
    const float dv = __uint_as_float(r[6]), va = __uint_as_float(r[7]), dx = __uint_as_float(r[8]);
    const unsigned long long iv = *reinterpret_cast<const unsigned long long *>(r + 10);
    const float vol = (float)((double)iv * 1e-18);
    const float t = tau < 1.0f ? 1.0f : tau;
    f[0] = log1pf(spread * h * K / margin);
    f[1] = log1pf(dv * K * K * h / (2.0f * t * margin));
    f[2] = vol / cell_vol;
    f[3] = tau / K;
    f[4] = log1pf(va * h * K / margin);
    f[5] = log1pf(dx / margin);
}

__global__ void __launch_bounds__(256) k_feat_predict(const uint32_t *raw, int64_t ncell, float h, float margin,
                                                     float tau, float K, float cell_vol, const float *params,
                                                     float *slot)
{
    __shared__ float sp[NPARAM];
    load_params(params, sp);
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float rr = 3.0e38f;
    if (c < ncell && raw[c * RAW + 3] != 0u) {
        float x[NF], h1[H], h2[H];
        feat_of_cell(raw + c * RAW, h, margin, tau, K, cell_vol, x);
        const float y = mlp_eval(sp, x, h1, h2);
        rr = expf(y) - 1.0f;
        if (!(rr >= 0.0f)) rr = 0.0f;
    }
    __shared__ float wmin[4];
    for (int d = 32; d > 0; d >>= 1) rr = fminf(rr, __shfl_xor(rr, d, 64));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = rr;
    __syncthreads();
    if (threadIdx.x == 0) slot[blockIdx.x] = fminf(fminf(wmin[0], wmin[1]), fminf(wmin[2], wmin[3]));
}

// Analytic interval: the largest n with (n + lambda) steps of motion at speed
// v plus gravity staying inside the margin, v t + g t^2 / 2 < m with
// t = (n + lambda) h; at least 1, at most kmax.
__device__ inline int64_t analytic_steps(const LearnedArgs &p, double v)
{
    double t;
    if (p.g > 0.0) t = (-v + sqrt(v * v + 2.0 * p.g * p.margin)) / p.g;
    else t = v > 0.0 ? p.margin / v : 1e30;
    const double n = floor(t / p.dt) - (double)p.lam;
    const int64_t k = n < 1.0 ? 1 : (n > 1e9 ? (int64_t)1e9 : (int64_t)n);
    return k < p.kmax ? k : p.kmax;
}

// The interval of the next work order, decided on the device: from the top
// speed of the last integration (blkmax, nblk slots) and the fastest point
// of any wall or mesh, the analytic bound (every geometry moves less than
// the margin); with a model, the minimum over cells of the predicted
// remaining steps (pslot, npslot slots), scaled by the safety factor, less
// the adoption latency and one step (the features see only the spheres:
// the analytic bound of the moving walls and meshes caps it; the analytic
// bound replaces it when no cell is occupied or the minimum is not finite).  out[0] = the interval, out[1] = the analytic bound, out[2] the
// bits of R (float).
__global__ void __launch_bounds__(256) k_learned_decide(const float *blkmax, int64_t nblk, const float *pslot,
                                                       int64_t npslot, LearnedArgs p, int64_t *out)
{
    float v2 = 0.0f, R = 3.0e38f;
    // eight independent loads in flight per thread
    const int64_t bs = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 7 * bs < nblk; i += 8 * bs) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = blkmax[i + k * bs];
#pragma unroll
        for (int k = 0; k < 8; ++k) v2 = fmaxf(v2, v[k]);
    }
    for (; i < nblk; i += bs) v2 = fmaxf(v2, blkmax[i]);
    for (i = threadIdx.x; i + 7 * bs < npslot; i += 8 * bs) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = pslot[i + k * bs];
#pragma unroll
        for (int k = 0; k < 8; ++k) R = fminf(R, v[k]);
    }
    for (; i < npslot; i += bs) R = fminf(R, pslot[i]);
    for (int d = 32; d > 0; d >>= 1) {
        v2 = fmaxf(v2, __shfl_xor(v2, d, 64));
        R = fminf(R, __shfl_xor(R, d, 64));
    }
    __shared__ float wv2[4], wr[4];
    if ((threadIdx.x & 63) == 0) {
        wv2[threadIdx.x >> 6] = v2;
        wr[threadIdx.x >> 6] = R;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    v2 = fmaxf(fmaxf(wv2[0], wv2[1]), fmaxf(wv2[2], wv2[3]));
    R = fminf(fminf(wr[0], wr[1]), fminf(wr[2], wr[3]));
    const double vmax = p.speed_valid && v2 == v2 ? sqrt((double)v2) : 0.0;
    const int64_t k_an = analytic_steps(p, fmax(vmax, p.vgeom));
    int64_t k = k_an;
    if (p.use_model && R >= 0.0f && R < 1.0e38f) {
        // R counts from the state the features saw, one step before the
        // work order (p.ahead = 1) or at it (0); the set is detected at the
        // order, adopted lambda steps later and used until the next set is
        // adopted k + lambda steps after the order, which must come before
        // the predicted first miss
        const double kl = floor(p.safety * (double)R) - (double)p.lam - 1.0 - (double)p.ahead;
        k = kl < 1.0 ? 1 : (int64_t)fmin(kl, 1e9);
        if (p.moving) {
            const int64_t km = analytic_steps(p, p.vgeom);
            k = k < km ? k : km;
        }
        k = k < p.kmax ? k : p.kmax;
    }
    out[0] = k;
    out[1] = k_an;
    out[2] = (int64_t)__float_as_uint(R);
}

__global__ void __launch_bounds__(256) k_snap_write(RecBuf rec, SnapRec *snap, int64_t No)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= No) return;
    const OwnerRec r = load_rec_hot(rec, o);
    SnapRec s;
    s.vox = r.vox;
    for (int k = 0; k < 3; ++k) {
        s.off[k] = r.off[k];
        s.v[k] = r.v[k];
    }
    snap[o] = s;
}

}  // namespace

// Feature pipeline used by both dem_features and the learned schedule:
// the per-cell accumulators of the owners' contributions (see k_feat_accum).
static void feature_accumulate(RecBuf rec, const SnapRec *snap, SnapRec *snap_out, const float *ovol,
                               Origin org, Grid fg, uint32_t *raw, uint32_t *cellmap, int64_t No, hipStream_t s)
{
    const int64_t nc = (int64_t)fg.nbins;
    hipLaunchKernelGGL(k_feat_clear, dim3(nblocks(nc * (RAW / 4), 256)), dim3(256), 0, s, raw, nc);
    const int64_t nb = (No + FEAT_OWNERS - 1) / FEAT_OWNERS;
    if (nb > 0)
        hipLaunchKernelGGL(k_feat_accum, dim3((unsigned)nb), dim3(256), 0, s, rec, snap, snap_out, ovol, org, fg, raw,
                           cellmap, No, stream_nt(No));
}

// Features of occupied cells written to `out` (row-major, cell order) and
// their count to pos[ncell]; cellmap[o] receives each owner's cell.
void feature_pipeline(RecBuf rec, const SnapRec *snap, const float *ovol, Origin org, Grid fg, float h,
                      float margin, float tau, uint32_t *raw, uint32_t *flags, uint32_t *pos, uint32_t *partials,
                      uint32_t *cellmap, float *out, uint32_t *cell_ids, int64_t No, hipStream_t s)
{
    int64_t nc = (int64_t)fg.nbins;
    feature_accumulate(rec, snap, nullptr, ovol, org, fg, raw, cellmap, No, s);
    hipLaunchKernelGGL(k_feat_flags, dim3(nblocks(nc, 256)), dim3(256), 0, s, raw, nc, flags);
    scan_exclusive_u32(flags, pos, nc, partials, s);
    double edge = 1.0 / fg.inv_b;
    float cell_vol = (float)(edge * edge * edge);
    hipLaunchKernelGGL(k_feat_write, dim3(nblocks(nc, 256)), dim3(256), 0, s, raw, pos, nc, h, margin, tau,
                       (float)DEM_MLP_KCAP, cell_vol, out, cell_ids);
}

// Slots of per-block prediction minima needed for ncell cells.
int64_t learned_slots(int64_t ncell)
{
    return (ncell + 255) / 256 + 1;
}

// The learned schedule's decision, all on the device (nothing read back
// here): with a model, the features of the current state against the
// snapshot (written over by the current state), the network on every
// occupied cell and the minimum of the predictions; then the interval
// (k_learned_decide) into out[0..2].
void learned_decide(RecBuf rec, SnapRec *snap, const float *ovol, Origin org, Grid fg, float h,
                    float margin, float tau, uint32_t *raw, const float *params, float *pslot, const float *blkmax,
                    int64_t nblk, const LearnedArgs &p, int64_t *out, int64_t No, hipStream_t s)
{
    const int64_t nc = (int64_t)fg.nbins;
    int64_t np = 0;
    if (p.use_model) {
        feature_accumulate(rec, snap, snap, ovol, org, fg, raw, nullptr, No, s);
        double edge = 1.0 / fg.inv_b;
        const float cell_vol = (float)(edge * edge * edge);
        np = (nc + 255) / 256;
        hipLaunchKernelGGL(k_feat_predict, dim3((unsigned)(np > 0 ? np : 1)), dim3(256), 0, s, raw, nc, h, margin,
                           tau, (float)DEM_MLP_KCAP, cell_vol, params, pslot);
    }
    hipLaunchKernelGGL(k_learned_decide, dim3(1), dim3(256), 0, s, blkmax, nblk, pslot, np, p, out);
}

void snapshot_write(RecBuf rec, SnapRec *snap, int64_t No, hipStream_t s)
{
    if (No > 0) hipLaunchKernelGGL(k_snap_write, dim3(nblocks(No, 256)), dim3(256), 0, s, rec, snap, No);
}

void mlp_forward(const float *params, const float *X, float *Y, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nblocks(n, 256)), dim3(256), 0, s, params, X, Y, n);
}


// Message of the last failed context-free call on this host thread
// (dem_last_error(NULL) returns it).
static thread_local std::string g_free_err;

const char *free_call_error()
{
    return g_free_err.c_str();
}

// Scratch of dem_mlp_backward_noalloc: the per-block partial gradients
// (NPARAM floats per block of BWD_SAMPLES samples) and partial losses (one
// float per block) of up to DEM_MLP_NOALLOC_MAX samples.  Every GPU the
// library runs on holds its own copy from the first kernel launch until the
// process ends.  In host code the array's name is not a device address: its
// address on each device comes from hipGetSymbolAddress (scratch_ptr).
constexpr int64_t NOALLOC_BLOCKS = DEM_MLP_NOALLOC_MAX / BWD_SAMPLES;
static_assert(NOALLOC_BLOCKS * BWD_SAMPLES == DEM_MLP_NOALLOC_MAX, "whole blocks");
static __device__ __align__(256) float scratch[NOALLOC_BLOCKS * NPARAM + NOALLOC_BLOCKS];

// The scratch's device address on the current device, looked up once per
// device (with that device current) and kept; nullptr on failure, with the
// reason in g_free_err.
static float *scratch_ptr()
{
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static float *ptr[MAX_DEV] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        g_free_err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    if (dev < 0 || dev >= MAX_DEV) {
        g_free_err = "device index out of range for the scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_free_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        ptr[dev] = static_cast<float *>(p);
    }
    return ptr[dev];
}

static void launch_backward(const float *params_dev, const float *X_dev, const float *T_dev, int64_t n, float tau,
                            float *grad_dev, float *loss_dev, float *partial, hipStream_t s)
{
    const int64_t nblk = (n + BWD_SAMPLES - 1) / BWD_SAMPLES;
    float *lpart = partial + nblk * NPARAM;
    hipLaunchKernelGGL(k_mlp_backward_block, dim3((unsigned)nblk), dim3(BWD_SAMPLES), 0, s, params_dev, X_dev, T_dev,
                       n, tau, partial, lpart);
    hipLaunchKernelGGL(k_mlp_backward_sum, dim3(nblocks(NPARAM + 1, 256)), dim3(256), 0, s, partial, lpart, nblk,
                       grad_dev, loss_dev);
}

extern "C" {

dem_status dem_mlp_forward(const float *params_dev, const float *X_dev, float *Y_dev, int64_t n, dem_stream stream)
{
    if (n < 0 || (n > 0 && (!params_dev || !X_dev || !Y_dev))) return DEM_ERR_ARG;
    mlp_forward(params_dev, X_dev, Y_dev, n, reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

int64_t dem_mlp_backward_work_bytes(int64_t n)
{
    int64_t nblk = (n + BWD_SAMPLES - 1) / BWD_SAMPLES;
    if (nblk < 1) nblk = 1;
    return (int64_t)sizeof(float) * (nblk * NPARAM + nblk) + 256;
}

dem_status dem_mlp_backward(const float *params_dev, const float *X_dev, const float *T_dev, int64_t n, float tau,
                            float *grad_dev, float *loss_dev, float *work_dev, int64_t work_bytes, dem_stream stream)
{
    if (n <= 0 || !params_dev || !X_dev || !T_dev || !grad_dev || !loss_dev || !work_dev) return DEM_ERR_ARG;
    if (work_bytes < dem_mlp_backward_work_bytes(n)) return DEM_ERR_ARG;
    if (!(tau > 0.0f && tau < 1.0f)) return DEM_ERR_ARG;
    launch_backward(params_dev, X_dev, T_dev, n, tau, grad_dev, loss_dev, work_dev,
                    reinterpret_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

dem_status dem_mlp_backward_noalloc(const float *params_dev, const float *X_dev, const float *T_dev, int64_t n,
                                    float tau, float *grad_dev, float *loss_dev, dem_stream stream)
{
    if (n <= 0 || !params_dev || !X_dev || !T_dev || !grad_dev || !loss_dev) {
        g_free_err = "dem_mlp_backward_noalloc: n must be > 0 and every pointer set";
        return DEM_ERR_ARG;
    }
    if (n > DEM_MLP_NOALLOC_MAX) {
        g_free_err = "dem_mlp_backward_noalloc: n = " + std::to_string(n) + " exceeds the scratch's " +
                     std::to_string((long long)DEM_MLP_NOALLOC_MAX) + " samples (use dem_mlp_backward)";
        return DEM_ERR_CAPACITY;
    }
    if (!(tau > 0.0f && tau < 1.0f)) {
        g_free_err = "dem_mlp_backward_noalloc: tau must lie in (0, 1)";
        return DEM_ERR_ARG;
    }
    float *p = scratch_ptr();
    if (!p) return DEM_ERR_HIP;
    // (every partial the sum reads is written first by its block: nothing
    // in the scratch needs clearing)
    launch_backward(params_dev, X_dev, T_dev, n, tau, grad_dev, loss_dev, p, reinterpret_cast<hipStream_t>(stream));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        g_free_err = std::string("dem_mlp_backward_noalloc launch: ") + hipGetErrorString(e);
        return DEM_ERR_HIP;
    }
    return DEM_OK;
}

dem_status dem_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int64_t t, float lr,
                        float beta1, float beta2, float eps, dem_stream stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev || t < 1) return DEM_ERR_ARG;
    float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_mlp_adam, dim3(nblocks(NPARAM, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       params_dev, grad_dev, m_dev, v_dev, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

}  // extern "C"
