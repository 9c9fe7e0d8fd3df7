// Learned contact-detection interval for gfx950.
//
// Features: per feature cell (a cube of 4 x 4 x 4 detection bins), from the
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
    if (i >= ncell) return;
    uint32_t *r = raw + i * RAW;
    for (int k = 0; k < 3; ++k) {
        r[k] = 0u;            // max of encoded v (encoded values are > 0)
        r[3 + k] = 0xffffffffu;  // min of encoded v
    }
    for (int k = 6; k < RAW; ++k) r[k] = 0u;
}

// Per-owner contributions to its feature cell.  Owners are numbered in
// space-filling order often enough that the lanes of a wave share few cells,
// so each wave first combines the values of its lanes per distinct cell
// (integer max / min / sums over shuffles, order-free) and one lane per
// cell issues the atomics.
__global__ void __launch_bounds__(256) k_feat_accum(const OwnerRec *rec, const OwnerRec *snap, const uint32_t *own_sph0,
                                                   const SphRec *sph, Origin org, Grid fg, uint32_t *raw,
                                                   uint32_t *cellmap, int64_t No)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = o < No;
    uint32_t c = 0xffffffffu;
    uint32_t vmax[3] = {0u, 0u, 0u}, vmin[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu};
    uint32_t fdv = 0u, fva = 0u, fdx = 0u, cnt = 0u;
    unsigned long long iv = 0ull;
    if (valid) {
        OwnerRec r = load_rec(rec + o);
        OwnerRec s = load_rec(snap + o);
        double X[3], Xs[3];
        for (int k = 0; k < 3; ++k) {
            X[k] = decode_axis(r.vox, r.off[k], org.o[k], k);
            Xs[k] = decode_axis(s.vox, s.off[k], org.o[k], k);
        }
        c = fcell_of(fg, X[0], X[1], X[2]);
        cellmap[o] = c;
        for (int k = 0; k < 3; ++k) {
            const uint32_t e = ord_enc(r.v[k]);
            vmax[k] = e;
            vmin[k] = e;
        }
        float dv0 = r.v[0] - s.v[0], dv1 = r.v[1] - s.v[1], dv2 = r.v[2] - s.v[2];
        float dv = sqrtf((dv0 * dv0 + dv1 * dv1) + dv2 * dv2);
        float va = sqrtf((r.v[0] * r.v[0] + r.v[1] * r.v[1]) + r.v[2] * r.v[2]);
        double d0 = X[0] - Xs[0], d1 = X[1] - Xs[1], d2 = X[2] - Xs[2];
        float dx = (float)sqrt((d0 * d0 + d1 * d1) + d2 * d2);
        fdv = __float_as_uint(dv);
        fva = __float_as_uint(va);
        fdx = __float_as_uint(dx);
        cnt = 1u;
        double vol = 0.0;
        for (uint32_t q = own_sph0[o]; q < own_sph0[o + 1]; ++q) {
            double rr = (double)sph[q].rad;
            vol += 4.18879020478639098 * rr * rr * rr;
        }
        // fixed-point volume in units of 1e-18 m^3
        iv = (unsigned long long)(vol * 1e18 + 0.5);
    }
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long todo = __ballot(valid);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const uint32_t cl = __shfl(c, leader, 64);
        const bool mine = valid && c == cl;
        const unsigned long long grp = __ballot(mine);
        uint32_t a[11];
        for (int k = 0; k < 3; ++k) {
            a[k] = mine ? vmax[k] : 0u;
            a[3 + k] = mine ? vmin[k] : 0xffffffffu;
        }
        a[6] = mine ? fdv : 0u;
        a[7] = mine ? fva : 0u;
        a[8] = mine ? fdx : 0u;
        a[9] = mine ? cnt : 0u;
        unsigned long long sv = mine ? iv : 0ull;
        for (int d = 32; d > 0; d >>= 1) {
            for (int k = 0; k < 3; ++k) {
                a[k] = max(a[k], (uint32_t)__shfl_xor(a[k], d, 64));
                a[3 + k] = min(a[3 + k], (uint32_t)__shfl_xor(a[3 + k], d, 64));
            }
            for (int k = 6; k < 9; ++k) a[k] = max(a[k], (uint32_t)__shfl_xor(a[k], d, 64));
            a[9] += (uint32_t)__shfl_xor(a[9], d, 64);
            sv += (unsigned long long)__shfl_xor((long long)sv, d, 64);
        }
        if (lane == leader) {
            uint32_t *rw = raw + (int64_t)cl * RAW;
            for (int k = 0; k < 3; ++k) {
                atomicMax(&rw[k], a[k]);
                atomicMin(&rw[3 + k], a[3 + k]);
            }
            atomicMax(&rw[6], a[6]);
            atomicMax(&rw[7], a[7]);
            atomicMax(&rw[8], a[8]);
            atomicAdd(&rw[9], a[9]);
            atomicAdd(reinterpret_cast<unsigned long long *>(&rw[10]), sv);
        }
        todo &= ~grp;
    }
}

__global__ void __launch_bounds__(256) k_feat_flags(const uint32_t *raw, int64_t ncell, uint32_t *flag)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    flag[c] = raw[c * RAW + 9] > 0u ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_feat_write(const uint32_t *raw, const uint32_t *pos, int64_t ncell,
                                                   float h, float margin, float tau, float K, float cell_vol,
                                                   float *out, uint32_t *cell_ids)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const uint32_t *r = raw + c * RAW;
    if (r[9] == 0u) return;
    uint32_t p = pos[c];
    float vr[3];
    for (int k = 0; k < 3; ++k) vr[k] = ord_dec(r[k]) - ord_dec(r[3 + k]);
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

// Minimum predicted remaining steps over cells: R = exp(y) - 1 (targets are
// log(1 + steps)), clamped at >= 0; order-free atomic minimum on float bits.
__global__ void __launch_bounds__(256) k_pred_min(const float *Y, int64_t n, uint32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float r = 3.0e38f;
    if (i < n) {
        float y = Y[i];
        r = expf(y) - 1.0f;
        if (!(r >= 0.0f)) r = 0.0f;
    }
    for (int d = 32; d > 0; d >>= 1) r = fminf(r, __shfl_xor(r, d, 64));
    if ((threadIdx.x & 63) == 0) atomicMin(out, __float_as_uint(r));
}

}  // namespace

// Feature pipeline used by both dem_features and the learned schedule.
// Writes features of occupied cells to `out` (row-major, cell order) and
// their count to `*ncell_dev`; cellmap[o] receives each owner's cell.
void feature_pipeline(const OwnerRec *rec, const OwnerRec *snap, const uint32_t *own_sph0, const SphRec *sph,
                      Origin org, Grid fg, float h, float margin, float tau, uint32_t *raw, uint32_t *flags,
                      uint32_t *pos, uint32_t *partials, uint32_t *cellmap, float *out, uint32_t *cell_ids,
                      int64_t No, hipStream_t s)
{
    int64_t nc = (int64_t)fg.nbins;
    hipLaunchKernelGGL(k_feat_clear, dim3(nblocks(nc, 256)), dim3(256), 0, s, raw, nc);
    hipLaunchKernelGGL(k_feat_accum, dim3(nblocks(No, 256)), dim3(256), 0, s, rec, snap, own_sph0, sph, org, fg,
                       raw, cellmap, No);
    hipLaunchKernelGGL(k_feat_flags, dim3(nblocks(nc, 256)), dim3(256), 0, s, raw, nc, flags);
    scan_exclusive_u32(flags, pos, nc, partials, s);
    double edge = 1.0 / fg.inv_b;
    float cell_vol = (float)(edge * edge * edge);
    hipLaunchKernelGGL(k_feat_write, dim3(nblocks(nc, 256)), dim3(256), 0, s, raw, pos, nc, h, margin, tau,
                       (float)DEM_MLP_KCAP, cell_vol, out, cell_ids);
}

void mlp_forward(const float *params, const float *X, float *Y, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nblocks(n, 256)), dim3(256), 0, s, params, X, Y, n);
}

void pred_min(const float *Y, int64_t n, uint32_t *out, hipStream_t s)
{
    launch_fill_u32(out, 1, 0x7f7fffffu, s);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_pred_min, dim3(nblocks(n, 256)), dim3(256), 0, s, Y, n, out);
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
