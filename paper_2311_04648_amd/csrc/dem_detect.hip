// Contact detection for gfx950 (paper Sec. 2.1: the active contact set is
// built with every geometry enlarged by a margin m).
//
//   bin:     sphere centres (exact FP64) -> bin key (uniform grid of cubic
//            bins of edge >= 2 (r_max + m), padded by one bin per side),
//            per-bin counts -> exclusive scan -> cell_start, and a sort of
//            (key, sphere id) by bin; candidate records are then gathered
//            into bin order so neighbour rows are contiguous.
//   detect:  one thread per sphere in bin order walks the forward half of
//            its 27-bin stencil and tests each candidate pair once with the
//            FP64 predicate |xi - xj|^2 < ((ri + rj) + 2m)^2 (after a
//            conservative FP32 prefilter), then the walls; a pair is staged
//            in the row of its lower id.  Facets of rigid meshes are walked
//            per facet over the bins near it (Sec. 2.4: a facet is one more
//            geometry) and staged in the sphere's row.  A scan of the row
//            counts gives the CSR offsets; each row is then sorted, so the
//            set is a list of ascending keys.
//   B lists: for every sphere, the contacts in which it is the higher id,
//            ascending; used by the ordered per-owner reduction.
//   remap:   per sphere, a merge of the old and the new row carries the
//            tangential history of surviving pairs; new pairs start at zero.
//   judge:   the full-stencil walk (and the facet walk) with m = 0 looks
//            every true contact up in the row of the set in use and counts
//            the missing ones.
#include "dem_device.h"

#include <algorithm>

namespace {

constexpr int TPB = 256;
constexpr int STAGE_K = 16;   // staged partners per sphere in the single-traversal detection

enum { MODE_COUNT = 0, MODE_WRITE = 1, MODE_JUDGE = 2, MODE_LABEL = 3 };

inline unsigned nblocks(int64_t n, int t = TPB)
{
    int64_t g = (n + t - 1) / t;
    return (unsigned)(g < 1 ? 1 : g);
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }


__global__ void __launch_bounds__(TPB) k_cd_prepare(DetectArgs a, uint32_t *keys, uint32_t *vals,
                                                    Cand *cand_tmp, uint32_t *cell_count, uint32_t *rank)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < a.n_spheres;
    if (!active) i = a.n_spheres - 1;   // the tail lanes take part in the wave's run claim only
    SphRec s = load_sph(a.sph + i);
    // a dormant sphere is not binned (it is found through the dormant
    // index): key nbins, no count, no slot in the sorted arrays
    const bool dorm = a.famdormant && a.famdormant[a.ofam[s.owner]];
    uint32_t key = a.grid.nbins;
    double x[3] = {0.0, 0.0, 0.0};
    if (!dorm) {
        const OwnerRec r = load_rec_hot(a.recs, s.owner);   // (the centre needs the hot part only)
        sphere_centre(r, s, a.q, a.tpos, a.org, x);
        key = bin_key(a.grid, x);
    }
    const uint32_t rk = wave_run_claim(cell_count, key, active && !dorm);
    if (a.nt) {
        // streams of a state larger than the caches: non-temporal stores,
        // the 32-byte candidate records through LDS so that each store
        // instruction writes 1 KiB of consecutive pieces (whole lines); a
        // dormant sphere's record (never read) is written too
        __shared__ uint4 lc[TPB / 64][128];
        const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
        lc[wv][2 * lane] = make_uint4(__double2loint(x[0]), __double2hiint(x[0]), __double2loint(x[1]),
                                      __double2hiint(x[1]));
        lc[wv][2 * lane + 1] = make_uint4(__double2loint(x[2]), __double2hiint(x[2]), __float_as_uint(s.rad),
                                          (uint32_t)i);
        if (active) {
            st_nt_u32(key, keys + i);
            if (vals) vals[i] = (uint32_t)i;
            if (!dorm) st_nt_u32(rk, rank + i);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t w0 = (int64_t)blockIdx.x * blockDim.x + 64 * wv;
        const uint32_t nv = w0 < a.n_spheres ? (uint32_t)(a.n_spheres - w0 < 64 ? a.n_spheres - w0 : 64) : 0u;
        uint4 *d = reinterpret_cast<uint4 *>(cand_tmp + w0);
        for (uint32_t k = lane; k < 2u * nv; k += 64u) st_nt(lc[wv][k], d + k);
        return;
    }
    if (!active) return;
    keys[i] = key;
    if (vals) vals[i] = (uint32_t)i;   // ids to sort (the one-pass sort writes its own)
    if (dorm) return;
    rank[i] = rk;
    Cand c;
    c.x = x[0];
    c.y = x[1];
    c.z = x[2];
    c.r = s.rad;
    c.id = (uint32_t)i;
    cand_tmp[i] = c;
}

// One-pass sort of (bin key, sphere id): the per-bin counts and their scan
// (the cell ranges) are the histogram and offsets of a single radix digit
// as wide as the key; each sphere's slot in its bin was claimed when the
// bins were counted (one atomic per run of equal keys in a wave), so the
// scatter writes each sphere at its bin's offset plus that slot, with no
// atomics; when asked each bin then orders its few ids ascending, so the
// result is identical to a stable sort.
__global__ void __launch_bounds__(TPB) k_bucket_scatter(const uint32_t *keys_in, const uint32_t *rank, int64_t n,
                                                        uint32_t nbins, const uint32_t *cell_start,
                                                        uint32_t *keys_out, uint32_t *vals_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = keys_in[i];
    if (k >= nbins) return;   // (key nbins: a dormant sphere, not binned)
    const uint32_t pos = cell_start[k] + rank[i];
    keys_out[pos] = k;
    vals_out[pos] = (uint32_t)i;
}

__global__ void __launch_bounds__(TPB) k_bucket_order(const uint32_t *cell_start, int64_t nbins, uint32_t *vals)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    uint32_t b0 = cell_start[b], b1 = cell_start[b + 1];
    for (uint32_t t = b0 + 1; t < b1; ++t) {
        uint32_t v = vals[t];
        uint32_t u = t;
        while (u > b0 && vals[u - 1] > v) {
            vals[u] = vals[u - 1];
            --u;
        }
        vals[u] = v;
    }
}

// Candidate records in bin order, and their 16-byte FP32 copies for the
// prefilter of the detection walk.
// (z1, z2: optional per-sphere counters of the detection that follows,
// n + 1 entries each, zeroed here rather than by a launch of their own)
__global__ void __launch_bounds__(TPB) k_cand_gather(const uint32_t *vals, const Cand *cand_tmp,
                                                     Cand *cand, float4 *candf, Grid g, int64_t n,
                                                     const uint32_t *cell_start, uint32_t *z1, uint32_t *z2, bool nt)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (z1 && p < n) {
        z1[p] = 0u;
        z2[p] = 0u;
        if (p == 0) {
            z1[n] = 0u;
            z2[n] = 0u;
        }
    }
    if (p >= n || p >= (int64_t)cell_start[g.nbins]) return;   // (dormant spheres sit after the binned ones)
    const Cand c = cand_tmp[vals[p]];
    if (cand) cand[p] = c;   // (null: no walk over bins reads the records in bin order)
    const float4 f = make_float4((float)(c.x - g.lo[0]), (float)(c.y - g.lo[1]), (float)(c.z - g.lo[2]), c.r);
    if (nt) st_nt(make_uint4(__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z), __float_as_uint(f.w)), reinterpret_cast<uint4 *>(candf + p));
    else candf[p] = f;
}

__device__ inline bool sphere_pair_hit(double xi, double yi, double zi, double ri, const Cand &cj,
                                       double m)
{
    double dx = xi - cj.x, dy = yi - cj.y, dz = zi - cj.z;
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double T = (ri + (double)cj.r) + 2.0 * m;
    return d2 < T * T;
}

__device__ inline bool wall_hit(const WallDev &w, const double *p, double x, double y, double z,
                                double r, double m)
{
    double rx = x - p[0], ry = y - p[1], rz = z - p[2];
    if (w.type == 0) {
        double sd = (rx * w.geom[3] + ry * w.geom[4]) + rz * w.geom[5];
        return sd < r + 2.0 * m;
    }
    double ax = (rx * w.geom[3] + ry * w.geom[4]) + rz * w.geom[5];
    double hl = 0.5 * w.geom[7] + 2.0 * m;
    if (!(ax <= hl && ax >= -hl)) return false;
    double px = rx - ax * w.geom[3], py = ry - ax * w.geom[4], pz = rz - ax * w.geom[5];
    double d2 = (px * px + py * py) + pz * pz;
    double T = (w.geom[6] + r) + 2.0 * m;
    return d2 < T * T;
}

// Whether contacts between the families of owners (or walls, meshes) fa and
// fb are listed.
__device__ inline bool fam_on(const DetectArgs &a, uint32_t fa, uint32_t fb)
{
    return !(a.pairoff && a.pairoff[256u * fa + fb]);
}

// Binary search of j in the ascending row [lo, hi) of a set.
__device__ inline bool row_contains(const uint32_t *row_j, uint32_t lo, uint32_t hi, uint32_t j)
{
    uint32_t a = lo, b = hi;
    while (a < b) {
        uint32_t mid = (a + b) >> 1;
        if (row_j[mid] < j) a = mid + 1;
        else b = mid;
    }
    return a < hi && row_j[a] == j;
}

// ---------------------------------------------------------------------------
// sphere-facet pairs
// ---------------------------------------------------------------------------
// Facets at the pose of one detection: world vertices, box, and the range of
// bins that holds every sphere centre within r_max + 2m of the box (grown by
// a rounding slack; bin_coord is monotone, so the clamped range is exact);
// frow[f] = the number of (y, z) bin rows of that range.
__global__ void __launch_bounds__(TPB) k_facet_prepare(DetectArgs a, FacetDev *fac, uint32_t *frow)
{
    const int32_t f = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (f >= a.n_tri) return;
    const TriDev t = a.tri[f];
    const MeshPose P = pose_of(a.poses, t.mesh);
    FacetDev d;
    facet_world(t, P, d.v);
    const double m = a.margin_dev ? *a.margin_dev : a.margin;
    const double e = (a.rmax + 2.0 * m) * (1.0 + 1e-9) + 1e-12;
    const int32_t nn[3] = {a.grid.nx, a.grid.ny, a.grid.nz};
    int c0[3], c1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double lo = fmin(d.v[k], fmin(d.v[3 + k], d.v[6 + k]));
        const double hi = fmax(d.v[k], fmax(d.v[3 + k], d.v[6 + k]));
        d.lo[k] = lo;
        d.hi[k] = hi;
        c0[k] = bin_coord(lo - e, a.grid.lo[k], a.grid.inv_b, nn[k]);
        c1[k] = bin_coord(hi + e, a.grid.lo[k], a.grid.inv_b, nn[k]);
        if (c1[k] < c0[k]) c1[k] = c0[k];   // NaN vertices: one bin, no pair passes the predicate
    }
    d.cx0 = c0[0];
    d.ncx = c1[0] - c0[0] + 1;
    d.cy0 = c0[1];
    d.ncy = c1[1] - c0[1] + 1;
    d.cz0 = c0[2];
    d.ncz = c1[2] - c0[2] + 1;
    d.family = P.family;
    d.pad[0] = d.pad[1] = d.pad[2] = 0;
    fac[f] = d;
    frow[f] = (uint32_t)d.ncy * (uint32_t)d.ncz;
}

// Box test before the exact predicate: rejects a centre farther than T (with
// slack) from the facet's box along one axis, which the exact predicate
// would reject too.
__device__ inline bool facet_box_near(const FacetDev &d, double x, double y, double z, double T)
{
    const double ts = T * (1.0 + 1e-9) + 1e-12;
    return !(x < d.lo[0] - ts || x > d.hi[0] + ts || y < d.lo[1] - ts || y > d.hi[1] + ts || z < d.lo[2] - ts ||
             z > d.hi[2] + ts);
}

// Sphere-facet predicate: |x - closest point|^2 < (r + 2m)^2 (strict).
__device__ inline bool facet_hit(const FacetDev &d, double x, double y, double z, double r, double m)
{
    const double T = r + 2.0 * m;
    if (!facet_box_near(d, x, y, z, T)) return false;
    const double p[3] = {x, y, z};
    double q[3];
    return facet_dist2(d.v, p, q) < T * T;
}

enum { FMODE_STAGE = 0, FMODE_JUDGE = 1, FMODE_LABEL = 2 };

// Sphere-facet pairs of one detection.  The (facet, bin row) pairs are
// numbered through the scanned frow; a wave takes 64 of them at a time (one
// per lane), concatenates the candidate ranges of its 64 rows with a wave
// prefix sum and tests the concatenation 64 candidates at a time (a lane
// finds the row of its candidate by a binary search over the lanes' running
// sums), so long and short rows, and large and small facets, spread evenly.
//   FMODE_STAGE: each pair joins the sphere's row like a wall (a slot of
//                `count` is claimed; the first STAGE_K are staged);
//   FMODE_JUDGE: each pair (m = 0) absent from the sphere's row of the set
//                in use adds one to *miss;
//   FMODE_LABEL: each such pair lowers first_miss of the sphere owner's cell
//                to tval.
template <int MODE>
__global__ void __launch_bounds__(TPB) k_facet_walk(DetectArgs a, const FacetDev *fac, const uint32_t *frow,
                                                    const Cand *cand, const uint32_t *cell_start, uint32_t *count,
                                                    uint32_t *stage, const uint32_t *cur_start,
                                                    const uint32_t *cur_j, int64_t cap, uint32_t *miss,
                                                    const uint32_t *cellmap, uint32_t *first_miss, uint32_t tval)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t nt = (uint32_t)a.n_tri;
    const uint32_t total = frow[nt];
    const double m = a.margin_dev ? *a.margin_dev : a.margin;
    const uint32_t nx = (uint32_t)a.grid.nx, ny = (uint32_t)a.grid.ny;
    const uint32_t jbase = (uint32_t)a.n_spheres + (uint32_t)a.n_walls;
    // rows of a set in use that overflowed its capacity are not valid
    const bool cur_ok = MODE != FMODE_STAGE && (int64_t)cur_start[a.n_spheres] <= cap;
    for (uint32_t r0 = wave * 64u; r0 < total; r0 += nwaves * 64u) {
        const uint32_t r = r0 + lane;
        uint32_t f = 0, s0 = 0, len = 0;
        if (r < total) {
            // the facet of row r: frow[f] <= r < frow[f + 1]
            uint32_t lo = 0, hi = nt;
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (frow[mid] <= r) lo = mid;
                else hi = mid;
            }
            f = lo;
            const FacetDev &d = fac[f];
            const uint32_t loc = r - frow[f];
            const uint32_t cy = (uint32_t)d.cy0 + loc % (uint32_t)d.ncy;
            const uint32_t cz = (uint32_t)d.cz0 + loc / (uint32_t)d.ncy;
            const uint32_t k0 = (cz * ny + cy) * nx + (uint32_t)d.cx0;
            s0 = cell_start[k0];
            len = cell_start[k0 + (uint32_t)d.ncx] - s0;
        }
        uint32_t inc = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o) inc += t;
        }
        const uint32_t tot = __shfl(inc, 63, 64);
        const uint32_t exc = inc - len;
        for (uint32_t vb = 0; vb < tot; vb += 64u) {
            const uint32_t v = vb + lane;
            // the lane whose range holds v: the number of lanes with inc <= v
            uint32_t k = 0;
#pragma unroll
            for (int st = 32; st >= 1; st >>= 1) {
                const uint32_t t = __shfl(inc, (int)(k + (uint32_t)st - 1u), 64);
                if (t <= v) k += (uint32_t)st;
            }
            const uint32_t fk = __shfl(f, (int)k, 64);
            const uint32_t sk = __shfl(s0, (int)k, 64);
            const uint32_t ek = __shfl(exc, (int)k, 64);
            if (v >= tot) continue;
            const Cand c = cand[sk + (v - ek)];
            if (!facet_hit(fac[fk], c.x, c.y, c.z, (double)c.r, m)) continue;
            if (a.pairoff && !fam_on(a, a.ofam[a.sph[c.id].owner], (uint32_t)fac[fk].family)) continue;
            const uint32_t jp = jbase + fk;
            if (MODE == FMODE_STAGE) {
                const uint32_t slot = atomicAdd(&count[c.id], 1u);
                if (slot < (uint32_t)STAGE_K) stage[(size_t)c.id * STAGE_K + slot] = jp;
            } else {
                const uint32_t lo_row = cur_ok ? cur_start[c.id] : 0u, hi_row = cur_ok ? cur_start[c.id + 1] : 0u;
                if (row_contains(cur_j, lo_row, hi_row, jp)) continue;
                if (MODE == FMODE_JUDGE) atomicAdd(miss, 1u);
                else atomicMin(&first_miss[cellmap[a.sph[c.id].owner]], tval);
            }
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(TPB) k_detect(DetectArgs a, const uint32_t *keys, const Cand *cand,
                                                const uint32_t *cell_start, uint32_t *count,
                                                const uint32_t *start, uint32_t *out_j, int64_t cap,
                                                const uint32_t *cur_start, const uint32_t *cur_j,
                                                uint32_t *miss, const uint32_t *cellmap = nullptr,
                                                uint32_t *first_miss = nullptr, uint32_t tval = 0)
{
    int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= a.n_spheres) return;
    const Cand ci = cand[p];
    const uint32_t i = ci.id;
    const uint32_t key = keys[p];
    const double xi = ci.x, yi = ci.y, zi = ci.z, ri = (double)ci.r;
    const double m = a.margin_dev ? *a.margin_dev : a.margin;
    const uint32_t nx = (uint32_t)a.grid.nx, nxy = (uint32_t)a.grid.nx * (uint32_t)a.grid.ny;
    uint32_t own_i = 0xffffffffu;
    uint32_t base = 0;
    bool can_write = true;
    if (MODE == MODE_WRITE) {
        base = start[i];
        can_write = (int64_t)start[i + 1] <= cap;
    }
    uint32_t lo_row = 0, hi_row = 0;
    if (MODE == MODE_JUDGE || MODE == MODE_LABEL) {
        // rows of a set that overflowed its capacity are not valid: treat as empty
        if ((int64_t)cur_start[a.n_spheres] <= cap) {
            lo_row = cur_start[i];
            hi_row = cur_start[i + 1];
        }
    }
    uint32_t n = 0, nmiss = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            uint32_t row = key + (uint32_t)((int)nxy * dz) + (uint32_t)((int)nx * dy);
            uint32_t q0 = cell_start[row - 1], q1 = cell_start[row + 2];
            for (uint32_t qq = q0; qq < q1; ++qq) {
                const Cand cj = cand[qq];
                if (cj.id <= i) continue;
                if (!sphere_pair_hit(xi, yi, zi, ri, cj, m)) continue;
                if (own_i == 0xffffffffu) own_i = a.sph[i].owner;
                const uint32_t own_j = a.sph[cj.id].owner;
                if (own_j == own_i) continue;
                if (a.pairoff && !fam_on(a, a.ofam[own_i], a.ofam[own_j])) continue;
                if (MODE == MODE_WRITE) {
                    if (can_write) out_j[base + n] = cj.id;
                } else if (MODE == MODE_JUDGE) {
                    if (!row_contains(cur_j, lo_row, hi_row, cj.id)) ++nmiss;
                } else if (MODE == MODE_LABEL) {
                    if (!row_contains(cur_j, lo_row, hi_row, cj.id)) {
                        atomicMin(&first_miss[cellmap[own_i]], tval);
                        atomicMin(&first_miss[cellmap[a.sph[cj.id].owner]], tval);
                    }
                }
                ++n;
            }
        }
    }
    // sort the sphere partners of this row (insertion sort, rows are short)
    if (MODE == MODE_WRITE && can_write) {
        for (uint32_t t = 1; t < n; ++t) {
            uint32_t v = out_j[base + t];
            uint32_t u = t;
            while (u > 0 && out_j[base + u - 1] > v) {
                out_j[base + u] = out_j[base + u - 1];
                --u;
            }
            out_j[base + u] = v;
        }
    }
    for (int w = 0; w < a.n_walls; ++w) {
        const WallDev wd = wall_at(a.walls, w);
        double pw[3];
        wall_point(wd, a.step, a.h, pw);
        if (!wall_hit(wd, pw, xi, yi, zi, ri, m)) continue;
        if (a.pairoff && !fam_on(a, a.ofam[a.sph[i].owner], (uint32_t)wd.family)) continue;
        uint32_t jp = (uint32_t)a.n_spheres + (uint32_t)w;
        if (MODE == MODE_WRITE) {
            if (can_write) out_j[base + n] = jp;
        } else if (MODE == MODE_JUDGE) {
            if (!row_contains(cur_j, lo_row, hi_row, jp)) ++nmiss;
        } else if (MODE == MODE_LABEL) {
            if (!row_contains(cur_j, lo_row, hi_row, jp)) atomicMin(&first_miss[cellmap[a.sph[i].owner]], tval);
        }
        ++n;
    }
    if (MODE == MODE_COUNT) count[i] = n;
    if (MODE == MODE_JUDGE && nmiss) atomicAdd(miss, nmiss);
}

// Single traversal over the forward half of the bin stencil: each sphere
// (in bin order) tests only the candidates after itself in its own bin and
// the 13 neighbour bins that follow its bin in key order -- bin x+1, the
// three bins of row y+1, the nine bins of plane z+1 -- so each pair of
// candidates is tested once.  The FP64 predicate is symmetric bit for bit.
// A pair found goes to the row of its lower id: the row's count is claimed
// with an atomic and the first STAGE_K partners are staged (their order is
// fixed later by sorting each row); the higher id's B-list count is bumped.
// Walls go to the sphere's own row.  `count` must be zero on entry.

// The FP32 prefilter of the detection walk (bound derived in
// k_detect_stage): true when candidate cj is farther from ci than the pair
// threshold by more than the rounding can account for.
__device__ inline bool prefilter_far(const float4 &ci, const float4 &cj, float Mi, float twom)
{
    const float dxf = ci.x - cj.x, dyf = ci.y - cj.y, dzf = ci.z - cj.z;
    const float Mj = fmaxf(fabsf(cj.x), fmaxf(fabsf(cj.y), fabsf(cj.z)));
    const float T32 = (ci.w + cj.w) + twom;
    const float tf = T32 + ((4.77e-7f * (Mi + Mj) + 9.54e-7f * T32) + 1e-12f);
    return (dxf * dxf + dyf * dyf) + dzf * dzf > tf * tf;
}

// Pairs of a binned sphere (bin `key`, FP32 copy cif, exact centre x, family
// fam_i) with the dormant spheres of the 27 bins around it, from the static
// dormant index; each pair that passes the exact predicate and is not
// switched off goes to f(dormant id).  A dormant sphere has no thread, so
// all its pairs with binned spheres are found here, whichever id is lower.
template <typename F>
__device__ inline void dormant_walk(const DetectArgs &a, uint32_t key, const float4 &cif, double xi, double yi,
                                    double zi, double ri, double m, uint32_t fam_i, F &&f)
{
    const float twom = (float)(2.0 * m);
    const float Mi = fmaxf(fabsf(cif.x), fmaxf(fabsf(cif.y), fabsf(cif.z)));
    const uint32_t nx = (uint32_t)a.grid.nx, nxy = (uint32_t)a.grid.nx * (uint32_t)a.grid.ny;
    for (int dz = -1; dz <= 1; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const uint32_t row = key + (uint32_t)((int)nxy * dz) + (uint32_t)((int)nx * dy);
            const uint32_t q1 = a.dcell_start[row + 2];
            for (uint32_t qq = a.dcell_start[row - 1]; qq < q1; ++qq) {
                if (prefilter_far(cif, a.dcandf[qq], Mi, twom)) continue;
                const Cand cj = a.dcand[qq];
                if (!sphere_pair_hit(xi, yi, zi, ri, cj, m)) continue;
                if (!fam_on(a, fam_i, a.ofam[a.sph[cj.id].owner])) continue;
                f(cj.id);
            }
        }
    }
}

// Whether sphere (FP32 copy cif relative to the grid origin, radius r)
// may be within the margin of wall w: the test of wall_hit on the centre
// recovered from its FP32 copy, with every threshold widened by the FP32
// rounding of that copy (each coordinate within 2^-24 M of the exact one,
// M its largest magnitude; 8 2^-24 M covers the three components through
// the projections) and 1e-9 m.  False means wall_hit is false.
__device__ inline bool wall_near(const WallDev &w, const double *p, const Grid &g, const float4 &cif, double r,
                                 double m)
{
    const double M = (double)fmaxf(fabsf(cif.x), fmaxf(fabsf(cif.y), fabsf(cif.z)));
    const double slack = 8.0 * 5.9604644775390625e-8 * M + 1e-9;
    const double rx = ((double)cif.x + g.lo[0]) - p[0], ry = ((double)cif.y + g.lo[1]) - p[1],
                 rz = ((double)cif.z + g.lo[2]) - p[2];
    if (w.type == 0) {
        const double sd = (rx * w.geom[3] + ry * w.geom[4]) + rz * w.geom[5];
        return sd < r + 2.0 * m + slack;
    }
    const double ax = (rx * w.geom[3] + ry * w.geom[4]) + rz * w.geom[5];
    const double hl = 0.5 * w.geom[7] + 2.0 * m + slack;
    if (!(ax <= hl && ax >= -hl)) return false;
    const double px = rx - ax * w.geom[3], py = ry - ax * w.geom[4], pz = rz - ax * w.geom[5];
    const double d2 = (px * px + py * py) + pz * pz;
    const double T = (w.geom[6] + r) + 2.0 * m + slack;
    return d2 < T * T;
}

// Sphere p of the bin order (id vals[p]) against the candidates after it
// in five contiguous ranges of the bin order (own bin after p and bin x+1;
// row y+1; rows y-1, y, y+1 of plane z+1).  The 64 spheres of a wave share
// one walk: their ranges are concatenated (a wave prefix sum of their
// counts; per sphere, in the wave's LDS slice, where each range ends in the
// concatenation and the offset that turns a concatenation index of the
// range into its bin-order position), and each round the wave takes the
// next 64 WALK_U candidates of the concatenation, one per lane and block of
// 64.  The sphere of a candidate is found without a search: each sphere
// whose candidates start in the round marks that slot (a byte per slot in
// LDS), and a lane takes the last mark at or before its slot (a ballot of
// the marked slots) or, with none, the sphere of the block's previous
// slot; so a wave runs as long as its spheres' mean candidate count, not
// its largest.  Per pair: an FP32 prefilter, then (clump systems) the
// candidate's id against the sphere range of the sphere's owner (spheres of
// one owner are consecutive and never a contact), then the exact FP64
// predicate on both exact centres, read by sphere id (cand_id), so the
// binning need not copy them into bin order.  Walls are prefiltered from
// the FP32 copy and each sphere's own lane tests them.
constexpr int WALK_U = 4;

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(TPB) k_detect_stage(DetectArgs a, const uint32_t *keys, const uint32_t *vals,
                                                      const Cand *cand_id, const float4 *candf,
                                                      const uint32_t *cell_start, uint32_t *count, uint32_t *stage,
                                                      uint32_t *bcount)
{
    // per wave and sphere lane: concatenation ends of ranges 0-3, position
    // offsets of ranges 0-4, FP32 copy, {largest coordinate of the copy,
    // owner's sphere range, sphere id}; per wave the start marks of a round
    __shared__ uint4 l_end[TPB / 64][64];
    __shared__ uint32_t l_off[TPB / 64][64 * 5];
    __shared__ float4 l_cif[TPB / 64][64];
    __shared__ uint4 l_aux[TPB / 64][64];
    __shared__ uint32_t l_mark[TPB / 64][64 * WALK_U / 4];
    const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // (dormant spheres are not binned: they sit after the binned ones; the
    // sphere's own loads are issued, in bounds, before that is known)
    const int64_t pc = p < a.n_spheres ? p : 0;
    const float4 cif_p = candf[pc];
    const uint32_t i_p = vals[pc], key_p = keys[pc];
    const bool valid = p < a.n_spheres && p < (int64_t)cell_start[a.grid.nbins];
    const double m = a.margin_dev ? *a.margin_dev : a.margin;
    const uint32_t nx = (uint32_t)a.grid.nx, nxy = (uint32_t)a.grid.nx * (uint32_t)a.grid.ny;
    float4 cif = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t i = 0, key = 0, total = 0, s0 = 0, s1 = 0;
    uint32_t ra[5] = {0u, 0u, 0u, 0u, 0u}, rl[5] = {0u, 0u, 0u, 0u, 0u};
    if (valid) {
        cif = cif_p;
        i = i_p;
        key = key_p;
        // (one load either way, so that it shares the round trip of the
        // bin ranges: without clumps a re-read of the sphere's own copy)
        const bool clumps = a.sph_range != nullptr;
        const uint2 sr = *(clumps ? a.sph_range + i : reinterpret_cast<const uint2 *>(candf + pc));
        s0 = clumps ? sr.x : i;
        s1 = clumps ? sr.y : i + 1u;
        const uint32_t e0 = cell_start[key + 2];
        ra[0] = (uint32_t)p + 1u;
        rl[0] = e0 - ra[0];
        const uint32_t r1 = key + nx;
        ra[1] = cell_start[r1 - 1];
        rl[1] = cell_start[r1 + 2] - ra[1];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const uint32_t row = key + nxy + (uint32_t)((int)nx * (t - 1));
            ra[2 + t] = cell_start[row - 1];
            rl[2 + t] = cell_start[row + 2] - ra[2 + t];
        }
        total = (rl[0] + rl[1]) + (rl[2] + rl[3] + rl[4]);
    }
    // the concatenation: exclusive prefix of the counts over the wave
    uint32_t inc = total;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)inc, d, 64);
        if ((int)lane >= d) inc += t;
    }
    const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    const uint32_t ex = inc - total;
    {
        // range k holds concatenation indices [c_k, c_k + rl[k]) and
        // bin-order positions ra[k] + (index - c_k): offset ra[k] - c_k
        // (modulo 2^32)
        uint32_t c = ex, e[4];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            l_off[wv][5 * lane + k] = ra[k] - c;
            c += rl[k];
            if (k < 4) e[k] = c;
        }
        l_end[wv][lane] = make_uint4(e[0], e[1], e[2], e[3]);
        l_cif[wv][lane] = cif;
        l_aux[wv][lane] = make_uint4(__float_as_uint(fmaxf(fabsf(cif.x), fmaxf(fabsf(cif.y), fabsf(cif.z)))), s0,
                                     s1, i);
    }
    // FP32 prefilter: a candidate is rejected only when its FP32 distance
    // exceeds the pair threshold T by more than a bound on the rounding.
    // Each FP32 coordinate is within 2^-24 |c| of the exact one (c: the
    // coordinate relative to the grid origin), so each difference is within
    // 2^-24 (M_i + M_j + |dx|) (M: largest coordinate magnitude of a sphere)
    // and the distance within sqrt(3) times that; the squares, sums and T
    // itself add a few 2^-24 relative.  The slack 8 2^-24 (M_i + M_j) +
    // 16 2^-24 T + 1e-12 m exceeds all of it, so no true pair is rejected;
    // the exact FP64 predicate decides the rest.
    const float twom = (float)(2.0 * m);
    const uint8_t *mark = reinterpret_cast<const uint8_t *>(l_mark[wv]);
    uint32_t carry = 0u;   // the sphere of the last slot of the block before
    for (uint32_t base = 0; base < T; base += 64u * WALK_U) {
        // start marks of the round (lane + 1; 0: no sphere starts here)
        wave_sync();
        l_mark[wv][lane] = 0u;
        wave_sync();
        if (total > 0u && ex >= base && ex - base < 64u * WALK_U)
            reinterpret_cast<uint8_t *>(l_mark[wv])[ex - base] = (uint8_t)(lane + 1u);
        wave_sync();
        uint32_t qb[WALK_U], jb[WALK_U], ob[WALK_U];
        float4 cb[WALK_U];
#pragma unroll
        for (int u = 0; u < WALK_U; ++u) {
            const uint32_t g0 = base + (uint32_t)u * 64u;
            const uint32_t g = g0 + lane;
            qb[u] = 0xffffffffu;
            ob[u] = 0u;
            if (g0 < T) {
                const uint32_t mk = mark[(uint32_t)u * 64u + lane];
                const uint64_t below = __ballot(mk != 0u) & (~0ull >> (63u - lane));
                uint32_t o = carry;
                if (below != 0ull) o = (uint32_t)mark[(uint32_t)u * 64u + (uint32_t)(63 - __clzll((long long)below))] - 1u;
                carry = (uint32_t)__builtin_amdgcn_readlane((int)o, 63);
                if (g < T) {
                    const uint4 e = l_end[wv][o];
                    const uint32_t r = (uint32_t)(g >= e.x) + (uint32_t)(g >= e.y) + (uint32_t)(g >= e.z) +
                                       (uint32_t)(g >= e.w);
                    qb[u] = g + l_off[wv][5u * o + r];
                    ob[u] = o;
                    cb[u] = candf[qb[u]];
                    jb[u] = vals[qb[u]];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < WALK_U; ++u) {
            if (qb[u] == 0xffffffffu) continue;
            const uint32_t o = ob[u];
            const float4 ci = l_cif[wv][o];
            const uint4 ax = l_aux[wv][o];
            const float dxf = ci.x - cb[u].x, dyf = ci.y - cb[u].y, dzf = ci.z - cb[u].z;
            const float Mj = fmaxf(fabsf(cb[u].x), fmaxf(fabsf(cb[u].y), fabsf(cb[u].z)));
            const float T32 = (ci.w + cb[u].w) + twom;
            const float tf = T32 + ((4.77e-7f * (__uint_as_float(ax.x) + Mj) + 9.54e-7f * T32) + 1e-12f);
            if ((dxf * dxf + dyf * dyf) + dzf * dzf > tf * tf) continue;
            const uint32_t j = jb[u];
            // (two spheres of one clump: never a contact)
            if (j >= ax.y && j < ax.z) continue;
            const uint32_t io = ax.w;
            const Cand c0 = cand_id[io];
            const Cand cj = cand_id[j];
            if (!sphere_pair_hit(c0.x, c0.y, c0.z, (double)ci.w, cj, m)) continue;
            if (a.pairoff && !fam_on(a, a.ofam[a.sph[io].owner], a.ofam[a.sph[j].owner])) continue;
            const uint32_t lo = io < j ? io : j, hi = io < j ? j : io;
            const uint32_t slot = atomicAdd(&count[lo], 1u);
            if (slot < (uint32_t)STAGE_K) stage[(size_t)lo * STAGE_K + slot] = hi;
            if (bcount) atomicAdd(&bcount[hi], 1u);
        }
    }
    if (!valid) return;
    // the sphere's own pairs with dormant spheres and walls
    const double ri = (double)cif.w;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    bool have_x = false;
    auto exact = [&]() {
        if (!have_x) {
            const Cand ci = cand_id[i];
            xi = ci.x;
            yi = ci.y;
            zi = ci.z;
            have_x = true;
        }
    };
    uint32_t own_i = 0xffffffffu;
    auto owner = [&]() {
        if (own_i == 0xffffffffu) own_i = a.sph[i].owner;
    };
    if (a.famdormant) {
        owner();
        exact();
        dormant_walk(a, key, cif, xi, yi, zi, ri, m, a.ofam[own_i], [&](uint32_t j) {
            const uint32_t lo = i < j ? i : j, hi = i < j ? j : i;
            const uint32_t slot = atomicAdd(&count[lo], 1u);
            if (slot < (uint32_t)STAGE_K) stage[(size_t)lo * STAGE_K + slot] = hi;
            if (bcount) atomicAdd(&bcount[hi], 1u);
        });
    }
    for (int w = 0; w < a.n_walls; ++w) {
        const WallDev wd = wall_at(a.walls, w);
        double pw[3];
        wall_point(wd, a.step, a.h, pw);
        if (!wall_near(wd, pw, a.grid, cif, ri, m)) continue;
        exact();
        if (!wall_hit(wd, pw, xi, yi, zi, ri, m)) continue;
        if (a.pairoff) {
            owner();
            if (!fam_on(a, a.ofam[own_i], (uint32_t)wd.family)) continue;
        }
        const uint32_t slot = atomicAdd(&count[i], 1u);
        if (slot < (uint32_t)STAGE_K) stage[(size_t)i * STAGE_K + slot] = (uint32_t)a.n_spheres + (uint32_t)w;
    }
}

// Appends sphere i to the B list of each sphere partner in its row.
__device__ inline void fill_blists(const uint32_t *row, uint32_t base, uint32_t n, uint32_t i, int64_t ns,
                                   uint32_t *bcur, uint32_t *bidx, uint32_t *bsrc)
{
    for (uint32_t t = 0; t < n; ++t) {
        const uint32_t jj = row[t];
        if ((int64_t)jj < ns) {
            const uint32_t slot = atomicAdd(&bcur[jj], 1u);
            bidx[slot] = base + t;
            bsrc[slot] = i;
        }
    }
}

// Moves staged rows (at most STAGE_K) to their CSR place, sorted, and fills
// the B lists (slot order is fixed later by k_blist_sort).  A row longer
// than STAGE_K is found again by a full-stencil walk for its sphere (its
// centre from the unsorted candidate records, its bin recomputed the same
// way as when binning), written, and sorted in place.
// (cand null: the candidates of the walk below are read by sphere id from
// cand_tmp, through the sorted ids vals)
__global__ void __launch_bounds__(TPB) k_compact(DetectArgs a, const Cand *cand_tmp, const Cand *cand,
                                                 const uint32_t *vals, const uint32_t *cell_start,
                                                 const uint32_t *start, const uint32_t *stage, uint32_t *out_j,
                                                 int64_t cap, uint32_t *bcur, uint32_t *bidx, uint32_t *bsrc,
                                                 const FacetDev *fac)
{
    const int64_t ns = a.n_spheres;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns || (int64_t)start[ns] > cap) return;
    const uint32_t r0 = start[i], n = start[i + 1] - r0;
    if (n == 0) return;
    if (n <= STAGE_K) {
        uint32_t v[STAGE_K];
        const uint32_t *st = stage + (size_t)i * STAGE_K;
#pragma unroll
        for (int t = 0; t < STAGE_K; ++t) v[t] = (uint32_t)t < n ? st[t] : 0xffffffffu;
        // sorting network on registers (odd-even transposition), ascending
#pragma unroll
        for (int r = 0; r < STAGE_K; ++r) {
#pragma unroll
            for (int t = (r & 1); t + 1 < STAGE_K; t += 2) {
                uint32_t lo = v[t] < v[t + 1] ? v[t] : v[t + 1];
                uint32_t hi = v[t] < v[t + 1] ? v[t + 1] : v[t];
                v[t] = lo;
                v[t + 1] = hi;
            }
        }
#pragma unroll
        for (int t = 0; t < STAGE_K; ++t) {
            if ((uint32_t)t < n) {
                out_j[r0 + t] = v[t];
                if (bidx && (int64_t)v[t] < ns) {
                    const uint32_t slot = atomicAdd(&bcur[v[t]], 1u);
                    bidx[slot] = r0 + t;
                    bsrc[slot] = (uint32_t)i;
                }
            }
        }
        return;
    }
    // the centre of sphere i: its candidate record, or for a dormant sphere
    // (not binned) its owner record, which does not change
    const uint32_t own_i = a.sph[i].owner;
    const bool dorm_i = a.famdormant && a.famdormant[a.ofam[own_i]];
    double xi, yi, zi, ri;
    if (dorm_i) {
        const SphRec si = load_sph(a.sph + i);
        double x[3];
        sphere_centre(load_rec_hot(a.recs, own_i), si, a.q, a.tpos, a.org, x);
        xi = x[0];
        yi = x[1];
        zi = x[2];
        ri = (double)si.rad;
    } else {
        const Cand ci = cand_tmp[i];
        xi = ci.x;
        yi = ci.y;
        zi = ci.z;
        ri = (double)ci.r;
    }
    const double m = a.margin_dev ? *a.margin_dev : a.margin;
    const int cx = bin_coord(xi, a.grid.lo[0], a.grid.inv_b, a.grid.nx);
    const int cy = bin_coord(yi, a.grid.lo[1], a.grid.inv_b, a.grid.ny);
    const int cz = bin_coord(zi, a.grid.lo[2], a.grid.inv_b, a.grid.nz);
    const uint32_t key = ((uint32_t)cz * (uint32_t)a.grid.ny + (uint32_t)cy) * (uint32_t)a.grid.nx + (uint32_t)cx;
    const uint32_t nx = (uint32_t)a.grid.nx, nxy = (uint32_t)a.grid.nx * (uint32_t)a.grid.ny;
    uint32_t *row = out_j + r0;
    uint32_t k = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        for (int dy = -1; dy <= 1; ++dy) {
            const uint32_t rw = key + (uint32_t)((int)nxy * dz) + (uint32_t)((int)nx * dy);
            const uint32_t q0 = cell_start[rw - 1], q1 = cell_start[rw + 2];
            for (uint32_t qq = q0; qq < q1; ++qq) {
                const Cand cj = cand ? cand[qq] : cand_tmp[vals[qq]];
                if (cj.id <= (uint32_t)i) continue;
                if (!sphere_pair_hit(xi, yi, zi, ri, cj, m)) continue;
                const uint32_t own_j = a.sph[cj.id].owner;
                if (own_j == own_i) continue;
                if (a.pairoff && !fam_on(a, a.ofam[own_i], a.ofam[own_j])) continue;
                if (k < n) row[k] = cj.id;
                ++k;
            }
        }
    }
    if (a.famdormant && !dorm_i) {
        const float4 cif = make_float4((float)(xi - a.grid.lo[0]), (float)(yi - a.grid.lo[1]),
                                       (float)(zi - a.grid.lo[2]), (float)ri);
        dormant_walk(a, key, cif, xi, yi, zi, ri, m, a.ofam[own_i], [&](uint32_t j) {
            if (j <= (uint32_t)i) return;
            if (k < n) row[k] = j;
            ++k;
        });
    }
    for (int w = 0; w < a.n_walls; ++w) {
        const WallDev wd = wall_at(a.walls, w);
        double pw[3];
        wall_point(wd, a.step, a.h, pw);
        if (!wall_hit(wd, pw, xi, yi, zi, ri, m)) continue;
        if (a.pairoff && !fam_on(a, a.ofam[own_i], (uint32_t)wd.family)) continue;
        if (k < n) row[k] = (uint32_t)ns + (uint32_t)w;
        ++k;
    }
    // facets: every facet's box, then the exact predicate (overflowing rows
    // are rare; the facet walk found the same pairs)
    for (int32_t f = 0; f < a.n_tri; ++f) {
        if (!facet_hit(fac[f], xi, yi, zi, ri, m)) continue;
        if (a.pairoff && !fam_on(a, a.ofam[own_i], (uint32_t)fac[f].family)) continue;
        if (k < n) row[k] = (uint32_t)ns + (uint32_t)a.n_walls + (uint32_t)f;
        ++k;
    }
    if (k > n) k = n;
    for (uint32_t t = 1; t < k; ++t) {
        const uint32_t v = row[t];
        uint32_t u = t;
        while (u > 0 && row[u - 1] > v) {
            row[u] = row[u - 1];
            --u;
        }
        row[u] = v;
    }
    if (bidx) fill_blists(row, r0, k, (uint32_t)i, ns, bcur, bidx, bsrc);
}

__global__ void k_check_capacity(const uint32_t *start, int64_t ns, int64_t cap, DevCounters *ctr,
                                 int buf)
{
    uint32_t total = start[ns];
    ctr->n_contacts[buf] = total;
    if ((int64_t)total > cap) {
        ctr->overflow[buf] = 1u;
        atomicMax(&ctr->required, total);
    } else {
        ctr->overflow[buf] = 0u;
    }
}

__global__ void k_record_total(const uint32_t *start, int64_t ns, DevCounters *ctr)
{
    ctr->required = start[ns];
}

__global__ void __launch_bounds__(TPB) k_blist_count(const uint32_t *start, const uint32_t *j,
                                                     int64_t ns, int64_t cap, uint32_t *bcount)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns || (int64_t)start[ns] > cap) return;   // an overflowed set has no valid rows
    for (uint32_t c = start[i]; c < start[i + 1]; ++c) {
        uint32_t jj = j[c];
        if ((int64_t)jj < ns) atomicAdd(&bcount[jj], 1u);
    }
}

__global__ void __launch_bounds__(TPB) k_blist_fill(const uint32_t *start, const uint32_t *j,
                                                    int64_t ns, int64_t cap, uint32_t *cursor, uint32_t *bidx,
                                                    uint32_t *bsrc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns || (int64_t)start[ns] > cap) return;
    for (uint32_t c = start[i]; c < start[i + 1]; ++c) {
        uint32_t jj = j[c];
        if ((int64_t)jj < ns) {
            const uint32_t slot = atomicAdd(&cursor[jj], 1u);
            bidx[slot] = c;
            bsrc[slot] = (uint32_t)i;
        }
    }
}

// Orders each B list by contact index (its source sphere moves along).
__global__ void __launch_bounds__(TPB) k_blist_sort(const uint32_t *start, const uint32_t *bstart, int64_t ns,
                                                    int64_t cap, uint32_t *bidx, uint32_t *bsrc)
{
    int64_t jv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (jv >= ns || (int64_t)start[ns] > cap) return;   // an overflowed set has no B lists
    uint32_t b0 = bstart[jv], b1 = bstart[jv + 1];
    for (uint32_t t = b0 + 1; t < b1; ++t) {
        const uint32_t v = bidx[t], w = bsrc[t];
        uint32_t u = t;
        while (u > b0 && bidx[u - 1] > v) {
            bidx[u] = bidx[u - 1];
            bsrc[u] = bsrc[u - 1];
            --u;
        }
        bidx[u] = v;
        bsrc[u] = w;
    }
}

// The last kernel of a detection: the B lists of sphere t sorted (as
// k_blist_sort), the flag of owner t (as k_owner_flags) and, striding over
// the bins, the bin counts zeroed for the next detection's front.
__global__ void __launch_bounds__(TPB) k_blist_finish(const uint32_t *start, const uint32_t *bstart, int64_t ns,
                                                      int64_t cap, uint32_t *bidx, uint32_t *bsrc,
                                                      const uint32_t *own_sph0, int64_t no, const uint8_t *ofam,
                                                      const uint8_t *fixed, uint8_t *flag, uint32_t *cell_count,
                                                      int64_t nz)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = t; k < nz; k += nthreads) cell_count[k] = 0u;
    const bool over = (int64_t)start[ns] > cap;
    if (t < ns && !over) {
        const uint32_t b0 = bstart[t], b1 = bstart[t + 1];
        for (uint32_t u0 = b0 + 1; u0 < b1; ++u0) {
            const uint32_t v = bidx[u0], w = bsrc[u0];
            uint32_t u = u0;
            while (u > b0 && bidx[u - 1] > v) {
                bidx[u] = bidx[u - 1];
                bsrc[u] = bsrc[u - 1];
                --u;
            }
            bidx[u] = v;
            bsrc[u] = w;
        }
    }
    if (t < no) {
        const uint8_t fx = (fixed && fixed[ofam[t]]) ? 2 : 0;
        if (over) {
            flag[t] = fx;
        } else {
            const uint32_t s0 = own_sph0 ? own_sph0[t] : (uint32_t)t;
            const uint32_t s1 = own_sph0 ? own_sph0[t + 1] : (uint32_t)t + 1u;
            flag[t] = (uint8_t)(((start[s0] != start[s1] || bstart[s0] != bstart[s1]) ? 1 : 0) | fx);
        }
    }
}

// Per-owner contact flag of a set: 1 if any sphere of owner o has a row or
// B-list entry (the spheres of an owner are consecutive, so their rows and
// B lists are one range each); an overflowed set flags nothing.
__global__ void __launch_bounds__(TPB) k_owner_flags(const uint32_t *start, const uint32_t *bstart,
                                                     const uint32_t *own_sph0, int64_t no, int64_t ns,
                                                     int64_t cap, const uint8_t *ofam, const uint8_t *fixed,
                                                     uint8_t *flag)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= no) return;
    const uint8_t fx = (fixed && fixed[ofam[o]]) ? 2 : 0;
    if ((int64_t)start[ns] > cap) {
        flag[o] = fx;
        return;
    }
    const uint32_t s0 = own_sph0 ? own_sph0[o] : (uint32_t)o;
    const uint32_t s1 = own_sph0 ? own_sph0[o + 1] : (uint32_t)o + 1u;
    flag[o] = (uint8_t)(((start[s0] != start[s1] || bstart[s0] != bstart[s1]) ? 1 : 0) | fx);
}

// The owners with contacts in a set, ascending: per tile of OL_TILE owners
// (OL_PER consecutive flags per thread, one 16-byte load) the count, a scan
// of the counts, then each tile writes its owners at its offset.
constexpr int OL_PER = 16;
constexpr int64_t OL_TILE = (int64_t)TPB * OL_PER;

__device__ inline uint32_t olist_bits(const uint8_t *flag, int64_t base, int64_t no)
{
    uint32_t bits = 0;
    if (base + OL_PER <= no) {
        const uint4 v = *reinterpret_cast<const uint4 *>(flag + base);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) bits |= ((w[k >> 2] >> (8 * (k & 3))) & 1u) << k;
    } else {
        for (int k = 0; k < OL_PER; ++k)
            if (base + k < no) bits |= (uint32_t)(flag[base + k] & 1u) << k;
    }
    return bits;
}

// exclusive prefix of v over the block (256 threads) and the block total
__device__ inline uint32_t olist_block_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t ws[TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) ws[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < TPB / 64; ++k) {
        off += k < wid ? ws[k] : 0u;
        tot += ws[k];
    }
    *total = tot;
    return inc - v + off;
}

__global__ void __launch_bounds__(TPB) k_olist_count(const uint8_t *flag, int64_t no, uint32_t *tcount)
{
    const int64_t base = (int64_t)blockIdx.x * OL_TILE + (int64_t)threadIdx.x * OL_PER;
    uint32_t tot;
    olist_block_scan((uint32_t)__popc(olist_bits(flag, base, no)), &tot);
    if (threadIdx.x == 0) tcount[blockIdx.x] = tot;
}

// Each listed owner's record carries its first sphere and the bounds of its
// spheres' rows and B lists (AcsBuf::olist), read here once per set so that
// the step reads them with the owner, in one sequential load.  The tile's
// listed owners are gathered in LDS first, then the block's threads take
// one each, so that a thread with several of them does not hold its wave.
__global__ void __launch_bounds__(TPB) k_olist_write(const uint8_t *flag, int64_t no, const uint32_t *toff,
                                                     const uint32_t *own_sph0, const uint32_t *start,
                                                     const uint32_t *bstart, uint4 *olist)
{
    __shared__ uint32_t lo[OL_TILE];
    const int64_t base = (int64_t)blockIdx.x * OL_TILE + (int64_t)threadIdx.x * OL_PER;
    uint32_t bits = olist_bits(flag, base, no), tot;
    uint32_t at = olist_block_scan((uint32_t)__popc(bits), &tot);
    while (bits) {
        lo[at++] = (uint32_t)(base + __ffs(bits) - 1);
        bits &= bits - 1u;
    }
    __syncthreads();
    const size_t pos0 = toff[blockIdx.x];
    for (uint32_t t = threadIdx.x; t < tot; t += TPB) {
        const uint32_t o = lo[t];
        const uint32_t s0 = own_sph0 ? own_sph0[o] : o, s1 = own_sph0 ? own_sph0[o + 1] : o + 1u;
        uint32_t n = s1 - s0;
        // every bound at once (up to s0 + LIST_SPHERES, and never past s1)
        uint32_t sb[LIST_SPHERES + 1], bb[LIST_SPHERES + 1];
#pragma unroll
        for (uint32_t m = 0; m <= LIST_SPHERES; ++m) {
            sb[m] = m <= n ? start[s0 + m] : 0u;
            bb[m] = m <= n ? bstart[s0 + m] : 0u;
        }
        uint64_t rows = 0, blist = 0;
        bool fits = n <= LIST_SPHERES;
#pragma unroll
        for (uint32_t m = 0; m < LIST_SPHERES; ++m)
            if (m < n) {
                const uint32_t na = sb[m + 1] - sb[m], nb = bb[m + 1] - bb[m];
                fits = fits && na <= 255u && nb <= 255u;
                rows |= (uint64_t)(na & 0xffu) << (8 * m);
                blist |= (uint64_t)(nb & 0xffu) << (8 * m);
            }
        if (!fits) n = LIST_NOPACK;
        olist[2 * (pos0 + t)] = make_uint4(o, s0, sb[0], bb[0]);
        olist[2 * (pos0 + t) + 1] = make_uint4((uint32_t)rows, (uint32_t)(rows >> 32) | (uint32_t)blist << 16,
                                               (uint32_t)(blist >> 16), n);
    }
}

__global__ void __launch_bounds__(TPB) k_remap(const uint32_t *os, const uint32_t *oj, const float *ohx,
                                               const float *ohy, const float *ohz, const float *ohw,
                                               const uint32_t *ns_, const uint32_t *nj, float *nhx, float *nhy,
                                               float *nhz, float *nhw, int64_t ns, DevCounters *ctr, int newbuf,
                                               int rolling)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (ctr->overflow[newbuf]) ctr->stop_cd = 1u;
    }
    if (i >= ns) return;
    if (ctr->overflow[newbuf]) return;
    uint32_t p = os[i], pe = os[i + 1];
    for (uint32_t c = ns_[i]; c < ns_[i + 1]; ++c) {
        uint32_t jj = nj[c];
        while (p < pe && oj[p] < jj) ++p;
        if (p < pe && oj[p] == jj) {
            nhx[c] = ohx[p];
            nhy[c] = ohy[p];
            nhz[c] = ohz[p];
            if (rolling) nhw[c] = ohw[p];
        } else {
            nhx[c] = 0.0f;
            nhy[c] = 0.0f;
            nhz[c] = 0.0f;
            if (rolling) nhw[c] = 0.0f;
        }
    }
}

// Static index of the dormant spheres: bin counts ...
__global__ void __launch_bounds__(TPB) k_dorm_count(DetectArgs a, uint32_t *dkey, uint32_t *dcount)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < a.n_spheres;
    if (!in) i = a.n_spheres - 1;
    const SphRec s = load_sph(a.sph + i);
    const bool dorm = in && a.famdormant[a.ofam[s.owner]];
    uint32_t key = 0;
    if (dorm) {
        double x[3];
        sphere_centre(load_rec_hot(a.recs, s.owner), s, a.q, a.tpos, a.org, x);
        const int cx = bin_coord(x[0], a.grid.lo[0], a.grid.inv_b, a.grid.nx);
        const int cy = bin_coord(x[1], a.grid.lo[1], a.grid.inv_b, a.grid.ny);
        const int cz = bin_coord(x[2], a.grid.lo[2], a.grid.inv_b, a.grid.nz);
        key = ((uint32_t)cz * (uint32_t)a.grid.ny + (uint32_t)cy) * (uint32_t)a.grid.nx + (uint32_t)cx;
        dkey[i] = key;
    }
    wave_run_claim(dcount, key, dorm);
}

// ... then the candidates, placed by a cursor per bin (order inside a bin
// is free: the pairs found do not depend on it).
__global__ void __launch_bounds__(TPB) k_dorm_fill(DetectArgs a, const uint32_t *dkey, uint32_t *dcursor, Cand *dcand,
                                                   float4 *dcandf)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i < a.n_spheres;
    if (!in) i = a.n_spheres - 1;
    const SphRec s = load_sph(a.sph + i);
    const bool dorm = in && a.famdormant[a.ofam[s.owner]];
    const uint32_t key = dorm ? dkey[i] : 0u;
    const uint32_t pos = wave_run_claim(dcursor, key, dorm);
    if (!dorm) return;
    double x[3];
    sphere_centre(load_rec_hot(a.recs, s.owner), s, a.q, a.tpos, a.org, x);
    Cand c;
    c.x = x[0];
    c.y = x[1];
    c.z = x[2];
    c.r = s.rad;
    c.id = (uint32_t)i;
    dcand[pos] = c;
    dcandf[pos] = make_float4((float)(c.x - a.grid.lo[0]), (float)(c.y - a.grid.lo[1]), (float)(c.z - a.grid.lo[2]),
                              c.r);
}

}  // namespace

void launch_dormant_index(const DetectArgs &a, CdWork &w, uint32_t *dcell_start, Cand *dcand, float4 *dcandf,
                          hipStream_t s)
{
    const int64_t n = a.n_spheres, nb = (int64_t)a.grid.nbins;
    launch_zero3(w.cell_count, nb + 1, nullptr, 0, nullptr, 0, s);
    hipLaunchKernelGGL(k_dorm_count, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys, w.cell_count);
    // bin ranges, with a copy as the fill cursor
    scan_exclusive_u32(w.cell_count, dcell_start, nb, w.partials, s, w.cell_count);
    hipLaunchKernelGGL(k_dorm_fill, dim3(nblocks(n)), dim3(TPB), 0, s, a, (const uint32_t *)w.keys, w.cell_count,
                       dcand, dcandf);
}

// First part of binning: zeroes the bin counts (and up to two further
// arrays of the caller in the same launch), then sphere centres, bin keys,
// unsorted candidate records and bin counts from the state in `a`.  After
// it, nothing of the binning reads the owner state.
void launch_bin_front(const DetectArgs &a, CdWork &w, hipStream_t s, uint32_t *z1, int64_t n1, uint32_t *z2,
                      int64_t n2)
{
    const int64_t n = a.n_spheres;
    launch_zero3(w.cell_count, (int64_t)a.grid.nbins + 1, z1, n1, z2, n2, s);
    hipLaunchKernelGGL(k_cd_prepare, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys,
                       w.sort_mode == 0 ? (uint32_t *)nullptr : w.vals, w.cand_tmp, w.cell_count, w.rank);
}

// Rest of binning: cell ranges, sort by bin, candidates in bin order.
// With `order_bins` the ids inside each bin are put in ascending order (a
// stable sort of (bin, id)); the detection does not need it: the pairs it
// finds do not depend on the order of the candidates inside a bin.
// With `bin_cand` false the candidate records are not copied into bin
// order (only their FP32 copies are written): the detection reads them by
// sphere id.
void launch_bin_back(const DetectArgs &a, CdWork &w, hipStream_t s, bool order_bins, uint32_t *z1 = nullptr,
                     uint32_t *z2 = nullptr, bool bin_cand = true)
{
    int64_t n = a.n_spheres;
    const int64_t nb = (int64_t)a.grid.nbins;
    if (w.sort_mode == 0) {
        // cell ranges; each sphere then goes to its bin's offset plus its slot
        scan_exclusive_u32(w.cell_count, w.cell_start, nb, w.partials, s);
        hipLaunchKernelGGL(k_bucket_scatter, dim3(nblocks(n)), dim3(TPB), 0, s, (const uint32_t *)w.keys,
                           (const uint32_t *)w.rank, n, a.grid.nbins, (const uint32_t *)w.cell_start, w.keys_alt,
                           w.vals_alt);
        if (order_bins)
            hipLaunchKernelGGL(k_bucket_order, dim3(nblocks(nb)), dim3(TPB), 0, s, w.cell_start, nb, w.vals_alt);
        uint32_t *t = w.keys; w.keys = w.keys_alt; w.keys_alt = t;
        t = w.vals; w.vals = w.vals_alt; w.vals_alt = t;
    } else {
        scan_exclusive_u32(w.cell_count, w.cell_start, nb, w.partials, s);
        radix_sort_u32(&w.keys, &w.vals, &w.keys_alt, &w.vals_alt, n, w.sort_bits, w.hist, w.partials, s);
    }
    // candidate records in bin order (random 32-byte reads, coalesced writes;
    // moving the records in the scatter instead costs more: random writes)
    hipLaunchKernelGGL(k_cand_gather, dim3(nblocks(n)), dim3(TPB), 0, s, w.vals, w.cand_tmp,
                       bin_cand ? w.cand : (Cand *)nullptr, w.candf, a.grid, n, (const uint32_t *)w.cell_start, z1,
                       z2, a.nt != 0);
}

void launch_bin(const DetectArgs &a, CdWork &w, hipStream_t s, uint32_t *z1, int64_t n1, uint32_t *z2,
                int64_t n2, bool order_bins)
{
    launch_bin_front(a, w, s, z1, n1, z2, n2);
    launch_bin_back(a, w, s, order_bins);
}

void launch_blists(AcsBuf &b, int64_t ns, int64_t cap, uint32_t *partials, hipStream_t s)
{
    launch_fill_u32(b.bcur, ns + 1, 0u, s);
    hipLaunchKernelGGL(k_blist_count, dim3(nblocks(ns)), dim3(TPB), 0, s, b.start, b.j, ns, cap, b.bcur);
    scan_exclusive_u32(b.bcur, b.bstart, ns, partials, s, b.bcur);
    hipLaunchKernelGGL(k_blist_fill, dim3(nblocks(ns)), dim3(TPB), 0, s, b.start, b.j, ns, cap, b.bcur, b.bidx,
                       b.bsrc);
    hipLaunchKernelGGL(k_blist_sort, dim3(nblocks(ns)), dim3(TPB), 0, s, b.start, b.bstart, ns, cap, b.bidx,
                       b.bsrc);
}

// Facets at the pose of the detection and the offsets of their bin rows.
void launch_facet_prepare(const DetectArgs &a, CdWork &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_facet_prepare, dim3(nblocks(a.n_tri)), dim3(TPB), 0, s, a, w.fac, w.frow);
    scan_exclusive_u32(w.frow, w.frow, a.n_tri, w.partials, s);
}

// The facet walk runs a fixed number of waves that stride over the rows.
inline unsigned facet_walk_blocks(const DetectArgs &a)
{
    return (unsigned)std::min<int64_t>(1024, std::max<int64_t>(64, ((int64_t)a.n_tri + 3) / 4));
}

// One kernel: the bin counts are zero on entry (left so by the back part),
// and the per-sphere counters are zeroed by the back part on its own
// stream, so the stream that owns the state runs no more than it must.
void launch_detect_front(const DetectArgs &a, CdWork &w, AcsBuf &out, hipStream_t s)
{
    hipLaunchKernelGGL(k_cd_prepare, dim3(nblocks(a.n_spheres)), dim3(TPB), 0, s, a, w.keys,
                       w.sort_mode == 0 ? (uint32_t *)nullptr : w.vals, w.cand_tmp, w.cell_count, w.rank);
}

int64_t owner_list_tiles(int64_t no)
{
    return (no + OL_TILE - 1) / OL_TILE;
}

void launch_owner_list(AcsBuf &b, const uint32_t *own_sph0, int64_t no, uint32_t *partials, hipStream_t s)
{
    const int64_t nt = owner_list_tiles(no);
    if (nt == 0) {
        launch_fill_u32(b.otile, 1, 0u, s);
        return;
    }
    hipLaunchKernelGGL(k_olist_count, dim3((unsigned)nt), dim3(TPB), 0, s, (const uint8_t *)b.oany, no, b.otile);
    scan_exclusive_u32(b.otile, b.otile, nt, partials, s);
    hipLaunchKernelGGL(k_olist_write, dim3((unsigned)nt), dim3(TPB), 0, s, (const uint8_t *)b.oany, no,
                       (const uint32_t *)b.otile, own_sph0, (const uint32_t *)b.start, (const uint32_t *)b.bstart,
                       b.olist);
}

void launch_owner_flags(AcsBuf &b, const uint32_t *own_sph0, int64_t no, int64_t ns, int64_t cap,
                        const uint8_t *ofam, const uint8_t *fixed, hipStream_t s, bool list, uint32_t *partials)
{
    hipLaunchKernelGGL(k_owner_flags, dim3(nblocks(no)), dim3(TPB), 0, s, (const uint32_t *)b.start,
                       (const uint32_t *)b.bstart, own_sph0, no, ns, cap, ofam, fixed, b.oany);
    if (list) launch_owner_list(b, own_sph0, no, partials, s);
}

void launch_detect(const DetectArgs &a, CdWork &w, AcsBuf &out, int64_t cap, DevCounters *ctr, int buf,
                   hipStream_t s)
{
    // (w may come from other uses that leave the bin counts set)
    launch_zero3(w.cell_count, (int64_t)a.grid.nbins + 1, nullptr, 0, nullptr, 0, s);
    launch_detect_front(a, w, out, s);
    launch_detect_back(a, w, out, cap, ctr, buf, s);
}

void launch_detect_back(const DetectArgs &a, CdWork &w, AcsBuf &out, int64_t cap, DevCounters *ctr, int buf,
                        hipStream_t s)
{
    int64_t n = a.n_spheres;
    // (the per-sphere counters out.bcur and w.count zeroed by the gather)
    // (the facet walk reads candidate records in bin order; without meshes
    // they are not copied)
    const bool bin_cand = a.n_tri > 0;
    launch_bin_back(a, w, s, false, out.bcur, w.count, bin_cand);
    hipLaunchKernelGGL(k_detect_stage, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys, w.vals, w.cand_tmp,
                       (const float4 *)w.candf, w.cell_start, w.count, w.stage, out.bcur);
    if (a.n_tri > 0) {
        launch_facet_prepare(a, w, s);
        hipLaunchKernelGGL(k_facet_walk<FMODE_STAGE>, dim3(facet_walk_blocks(a)), dim3(TPB), 0, s, a,
                           (const FacetDev *)w.fac, (const uint32_t *)w.frow, (const Cand *)w.cand,
                           (const uint32_t *)w.cell_start, w.count, w.stage, (const uint32_t *)nullptr,
                           (const uint32_t *)nullptr, cap, (uint32_t *)nullptr, (const uint32_t *)nullptr,
                           (uint32_t *)nullptr, 0u);
    }
    // row offsets (checked against the capacity) and B-list offsets (with a
    // copy as the fill cursor) in one pair of launches
    scan_exclusive_u32_pair(w.count, out.start, nullptr, ctr, cap, buf, out.bcur, out.bstart, out.bcur, n,
                            w.partials, s);
    hipLaunchKernelGGL(k_compact, dim3(nblocks(n)), dim3(TPB), 0, s, a, (const Cand *)w.cand_tmp,
                       bin_cand ? (const Cand *)w.cand : (const Cand *)nullptr, (const uint32_t *)w.vals,
                       (const uint32_t *)w.cell_start, (const uint32_t *)out.start, (const uint32_t *)w.stage, out.j,
                       cap, out.bcur, out.bidx, out.bsrc, (const FacetDev *)w.fac);
    // B lists sorted, owner flags, and the bin counts (dead since the
    // scatter) zeroed for the next front, in one launch
    hipLaunchKernelGGL(k_blist_finish, dim3(nblocks(std::max(n, a.n_owners))), dim3(TPB), 0, s, out.start,
                       out.bstart, n, cap, out.bidx, out.bsrc, a.own_sph0, a.n_owners, a.ofam, a.famfixed, out.oany,
                       w.cell_count, (int64_t)a.grid.nbins + 1);
    if (a.owner_list) launch_owner_list(out, a.own_sph0, a.n_owners, w.partials, s);
}

void launch_judge(const DetectArgs &a_in, CdWork &w, const AcsBuf &cur, int64_t cap, DevCounters *ctr,
                  hipStream_t s)
{
    // every sphere binned: the judge's full-stencil walk finds each pair from its lower id
    DetectArgs a = a_in;
    a.famdormant = nullptr;
    int64_t n = a.n_spheres;
    launch_bin(a, w, s, nullptr, 0, nullptr, 0, false);
    hipLaunchKernelGGL(k_detect<MODE_JUDGE>, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys, w.cand,
                       w.cell_start, (uint32_t *)nullptr, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                       cap, (const uint32_t *)cur.start, (const uint32_t *)cur.j, &ctr->miss,
                       (const uint32_t *)nullptr, (uint32_t *)nullptr, 0u);
    if (a.n_tri > 0) {
        launch_facet_prepare(a, w, s);
        hipLaunchKernelGGL(k_facet_walk<FMODE_JUDGE>, dim3(facet_walk_blocks(a)), dim3(TPB), 0, s, a,
                           (const FacetDev *)w.fac, (const uint32_t *)w.frow, (const Cand *)w.cand,
                           (const uint32_t *)w.cell_start, (uint32_t *)nullptr, (uint32_t *)nullptr,
                           (const uint32_t *)cur.start, (const uint32_t *)cur.j, cap, &ctr->miss,
                           (const uint32_t *)nullptr, (uint32_t *)nullptr, 0u);
    }
}

void launch_remap(const AcsBuf &o, AcsBuf &nb, int64_t ns, DevCounters *ctr, int newbuf, int rolling,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_remap, dim3(nblocks(ns)), dim3(TPB), 0, s, o.start, o.j, o.hx, o.hy, o.hz, o.hw,
                       nb.start, nb.j, nb.hx, nb.hy, nb.hz, nb.hw, ns, ctr, newbuf, rolling);
}

void launch_detect_plain(const DetectArgs &a_in, CdWork &w, uint32_t *start, uint32_t *j, int64_t cap,
                         DevCounters *ctr, hipStream_t s)
{
    DetectArgs a = a_in;
    a.famdormant = nullptr;
    int64_t n = a.n_spheres;
    launch_bin(a, w, s, w.count, n + 1, nullptr, 0, false);
    hipLaunchKernelGGL(k_detect_stage, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys, w.vals, w.cand_tmp,
                       (const float4 *)w.candf, w.cell_start, w.count, w.stage, (uint32_t *)nullptr);
    if (a.n_tri > 0) {
        launch_facet_prepare(a, w, s);
        hipLaunchKernelGGL(k_facet_walk<FMODE_STAGE>, dim3(facet_walk_blocks(a)), dim3(TPB), 0, s, a,
                           (const FacetDev *)w.fac, (const uint32_t *)w.frow, (const Cand *)w.cand,
                           (const uint32_t *)w.cell_start, w.count, w.stage, (const uint32_t *)nullptr,
                           (const uint32_t *)nullptr, cap, (uint32_t *)nullptr, (const uint32_t *)nullptr,
                           (uint32_t *)nullptr, 0u);
    }
    scan_exclusive_u32(w.count, start, n, w.partials, s);
    hipLaunchKernelGGL(k_record_total, dim3(1), dim3(1), 0, s, start, n, ctr);
    hipLaunchKernelGGL(k_compact, dim3(nblocks(n)), dim3(TPB), 0, s, a, (const Cand *)w.cand_tmp,
                       (const Cand *)w.cand, (const uint32_t *)w.vals, (const uint32_t *)w.cell_start,
                       (const uint32_t *)start, (const uint32_t *)w.stage, j, cap, (uint32_t *)nullptr,
                       (uint32_t *)nullptr, (uint32_t *)nullptr, (const FacetDev *)w.fac);
}

void launch_label_judge(const DetectArgs &a_in, CdWork &w, const uint32_t *lab_start, const uint32_t *lab_j,
                        int64_t cap, const uint32_t *cellmap, uint32_t *first_miss, uint32_t tval,
                        hipStream_t s)
{
    DetectArgs a = a_in;
    a.famdormant = nullptr;
    int64_t n = a.n_spheres;
    launch_bin(a, w, s, nullptr, 0, nullptr, 0, false);
    hipLaunchKernelGGL(k_detect<MODE_LABEL>, dim3(nblocks(n)), dim3(TPB), 0, s, a, w.keys, w.cand,
                       w.cell_start, (uint32_t *)nullptr, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                       cap, lab_start, lab_j, (uint32_t *)nullptr, cellmap, first_miss, tval);
    if (a.n_tri > 0) {
        launch_facet_prepare(a, w, s);
        hipLaunchKernelGGL(k_facet_walk<FMODE_LABEL>, dim3(facet_walk_blocks(a)), dim3(TPB), 0, s, a,
                           (const FacetDev *)w.fac, (const uint32_t *)w.frow, (const Cand *)w.cand,
                           (const uint32_t *)w.cell_start, (uint32_t *)nullptr, (uint32_t *)nullptr, lab_start,
                           lab_j, cap, (uint32_t *)nullptr, cellmap, first_miss, tval);
    }
}
