// Device (and host) helpers: position codec, rotations, small vector math.
// Every FP64 expression that decides a contact predicate is written with an
// explicit operation order; the library is compiled with -ffp-contract=off
// so no multiply-add is fused and each operation rounds once.
#pragma once

#include "dem_internal.h"

// ---------------------------------------------------------------------------
// position codec: world X = origin + vox * 2^-14 + off, off on a 2^-38 grid.
// Every value of this form is an FP64 number, so decoding is exact.
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t vox_axis(uint64_t vox, int k)
{
    return (uint32_t)((vox >> (DEM_VOX_BITS * k)) & DEM_VOX_MASK);
}

__host__ __device__ inline double decode_axis(uint64_t vox, float off, double origin, int k)
{
    double local = (double)vox_axis(vox, k) * DEM_VOXEL_SIZE + (double)off;
    return origin + local;
}

// Encodes one axis of a world coordinate.  Rounds to the nearest 2^-38 m.
__host__ __device__ inline void encode_axis(double x, double origin, uint32_t *iv, float *off)
{
    double local = x - origin;
    double v = floor(local * DEM_VOXEL_INV);
    if (!(v >= 0.0)) v = 0.0;                      // also catches NaN
    if (v > (double)DEM_VOX_MASK) v = (double)DEM_VOX_MASK;
    double r = local - v * DEM_VOXEL_SIZE;
    double kq = rint(r * DEM_OFF_QUANT_INV);
    if (kq < 0.0) kq = 0.0;
    if (kq >= DEM_OFF_STEPS) {
        if (v < (double)DEM_VOX_MASK) {
            v += 1.0;
            kq = 0.0;
        } else {
            kq = DEM_OFF_STEPS - 1.0;
        }
    }
    *iv = (uint32_t)v;
    *off = (float)(kq * DEM_OFF_QUANT);
}

// The top bit of an owner record's voxel word (the three axes use the
// low 63 bits; pack_vox leaves it clear): set by the streaming clump step
// when both orientation buffers hold the owner's orientation, so that a
// clump at rest on that path needs neither read nor write of it.  Every
// other writer of a record clears it (pack_vox) or copies both buffers.
constexpr uint64_t DEM_VOX_QSAME = 1ull << 63;

__host__ __device__ inline uint64_t pack_vox(uint32_t x, uint32_t y, uint32_t z)
{
    return (uint64_t)x | ((uint64_t)y << DEM_VOX_BITS) | ((uint64_t)z << (2 * DEM_VOX_BITS));
}

// ---------------------------------------------------------------------------
// rotation of a unit quaternion (w,x,y,z), body -> world, fixed formula
// ---------------------------------------------------------------------------
struct Mat3d {
    double m[9];
};

__host__ __device__ inline Mat3d rot_from_q(double w, double x, double y, double z)
{
    Mat3d R;
    R.m[0] = 1.0 - 2.0 * (y * y + z * z);
    R.m[1] = 2.0 * (x * y - w * z);
    R.m[2] = 2.0 * (x * z + w * y);
    R.m[3] = 2.0 * (x * y + w * z);
    R.m[4] = 1.0 - 2.0 * (x * x + z * z);
    R.m[5] = 2.0 * (y * z - w * x);
    R.m[6] = 2.0 * (x * z - w * y);
    R.m[7] = 2.0 * (y * z + w * x);
    R.m[8] = 1.0 - 2.0 * (x * x + y * y);
    return R;
}

__host__ __device__ inline void rot_apply(const Mat3d &R, double px, double py, double pz, double *o)
{
    o[0] = (R.m[0] * px + R.m[1] * py) + R.m[2] * pz;
    o[1] = (R.m[3] * px + R.m[4] * py) + R.m[5] * pz;
    o[2] = (R.m[6] * px + R.m[7] * py) + R.m[8] * pz;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  This maps the dispatch index to a logical block so that every XCD
// works on one contiguous range of blocks: neighbouring spheres (which share
// neighbour rows and partner records) then meet in the same L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t n)
{
    const uint32_t per = n >> 3, rem = n & 7u, x = b & 7u, k = b >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

// Claims one slot of counter[key] per active lane (key < 2^32 - 1): lanes
// of a run of equal keys in consecutive active lanes share one atomic,
// issued by the run's first lane with the run's length; returns each
// lane's slot (the counter's old value plus its rank in the run).  Spheres
// numbered in space-filling order put runs of neighbours in one bin, whose
// atomics would otherwise serialise on one address.
__device__ inline uint32_t wave_run_claim(uint32_t *counter, uint32_t key_in, bool active)
{
    const int lane = (int)(threadIdx.x & 63u);
    const uint32_t key = active ? key_in : 0xffffffffu;   // an inactive lane ends a run
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool head = active && (lane == 0 || prev != key);
    const unsigned long long heads = __ballot(head), act = __ballot(active);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0 .. lane
    const unsigned long long hb = heads & upto;
    const int h = hb ? 63 - __clzll((long long)hb) : 0;
    uint32_t base = 0;
    if (head) {
        const unsigned long long above = (heads | ~act) & ~upto;   // next head or first inactive lane
        const int next = above ? __ffsll((long long)above) - 1 : 64;
        base = atomicAdd(&counter[key], (uint32_t)(next - lane));
    }
    base = __shfl(base, h, 64);
    return base + (uint32_t)(lane - h);
}

__device__ inline float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ inline float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ inline float dot3(float3 a, float3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ inline float3 cross3(float3 a, float3 b)
{
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// An owner record from its hot part (a, b) and cold part (c).
__device__ inline OwnerRec rec_from(uint4 a, uint4 b, uint4 c)
{
    OwnerRec r;
    r.vox = (uint64_t)a.x | ((uint64_t)a.y << 32);
    r.off[0] = __uint_as_float(a.z);
    r.off[1] = __uint_as_float(a.w);
    r.off[2] = __uint_as_float(b.x);
    r.v[0] = __uint_as_float(b.y);
    r.v[1] = __uint_as_float(b.z);
    r.v[2] = __uint_as_float(b.w);
    r.w[0] = __uint_as_float(c.x);
    r.w[1] = __uint_as_float(c.y);
    r.w[2] = __uint_as_float(c.z);
    r.mass = __uint_as_float(c.w);
    return r;
}

__device__ inline uint4 rec_hot0(const OwnerRec &r)
{
    return make_uint4((uint32_t)r.vox, (uint32_t)(r.vox >> 32), __float_as_uint(r.off[0]), __float_as_uint(r.off[1]));
}

__device__ inline uint4 rec_hot1(const OwnerRec &r)
{
    return make_uint4(__float_as_uint(r.off[2]), __float_as_uint(r.v[0]), __float_as_uint(r.v[1]),
                      __float_as_uint(r.v[2]));
}

__device__ inline uint4 rec_cold(const OwnerRec &r)
{
    return make_uint4(__float_as_uint(r.w[0]), __float_as_uint(r.w[1]), __float_as_uint(r.w[2]),
                      __float_as_uint(r.mass));
}

// Owner o's record: three 16-byte loads.  Two layouts (RecBuf): clump
// systems keep hot and cold parts in two arrays; single-sphere systems
// (cold null) whole 48-byte records in one array, three uint4 per owner.
__device__ inline OwnerRec load_rec(const RecBuf &b, int64_t o)
{
    if (b.cold) return rec_from(b.hot[2 * o], b.hot[2 * o + 1], b.cold[o]);
    return rec_from(b.hot[3 * o], b.hot[3 * o + 1], b.hot[3 * o + 2]);
}

// Its hot part only (position and velocity; w and mass read as zero).
__device__ inline OwnerRec load_rec_hot(const RecBuf &b, int64_t o)
{
    const int64_t k = (b.cold ? 2 : 3) * o;
    return rec_from(b.hot[k], b.hot[k + 1], make_uint4(0u, 0u, 0u, 0u));
}

// Its cold part into r (w, mass).
__device__ inline void load_rec_cold(const RecBuf &b, int64_t o, OwnerRec &r)
{
    const uint4 c = b.cold ? b.cold[o] : b.hot[3 * o + 2];
    r.w[0] = __uint_as_float(c.x);
    r.w[1] = __uint_as_float(c.y);
    r.w[2] = __uint_as_float(c.z);
    r.mass = __uint_as_float(c.w);
}

__device__ inline void store_rec(const RecBuf &b, int64_t o, const OwnerRec &r)
{
    const int64_t k = (b.cold ? 2 : 3) * o;
    b.hot[k] = rec_hot0(r);
    b.hot[k + 1] = rec_hot1(r);
    if (b.cold) b.cold[o] = rec_cold(r);
    else b.hot[k + 2] = rec_cold(r);
}

__device__ inline void store_rec_hot(const RecBuf &b, int64_t o, const OwnerRec &r)
{
    const int64_t k = (b.cold ? 2 : 3) * o;
    b.hot[k] = rec_hot0(r);
    b.hot[k + 1] = rec_hot1(r);
}

// The same for split records (clump systems) only: no layout test.
// Stores of streams that no kernel reads back soon enough for a cache to
// serve it (whole arrays larger than the caches): non-temporal, so they do
// not evict data that is reused.
typedef unsigned int u32x4_nt __attribute__((ext_vector_type(4)));
__device__ inline void st_nt(uint4 v, uint4 *p)
{
    const u32x4_nt w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4_nt *>(p));
}

__device__ inline void st_nt_u32(uint32_t v, uint32_t *p)
{
    __builtin_nontemporal_store(v, p);
}

__device__ inline OwnerRec load_split_hot(const RecBuf &b, int64_t o)
{
    return rec_from(b.hot[2 * o], b.hot[2 * o + 1], make_uint4(0u, 0u, 0u, 0u));
}

// (nt: the streaming step's output of a state larger than the caches, read
// back a whole array later)
__device__ inline void store_split_hot(const RecBuf &b, int64_t o, const OwnerRec &r, bool nt)
{
    if (nt) {
        st_nt(rec_hot0(r), &b.hot[2 * o]);
        st_nt(rec_hot1(r), &b.hot[2 * o + 1]);
    } else {
        b.hot[2 * o] = rec_hot0(r);
        b.hot[2 * o + 1] = rec_hot1(r);
    }
}

// A wave's 64 records in LDS (192 uint4) in the layout of `like`.
__device__ inline RecBuf rec_lds(uint4 *buf, const RecBuf &like)
{
    return RecBuf{buf, like.cold ? buf + 128 : nullptr};
}

// One wave copies the records of n owners, from src owner s0 to dst owner
// d0 (global memory or LDS, both in one layout): their hot parts, and
// their cold parts if `cold` (whole records are copied where they are not
// split).
__device__ inline void rec_copy(const RecBuf &dst, int64_t d0, const RecBuf &src, int64_t s0, uint32_t n,
                                uint32_t lane, bool cold)
{
    if (!src.cold) {
        for (uint32_t k = lane; k < 3u * n; k += 64u) dst.hot[3 * d0 + k] = src.hot[3 * s0 + k];
        return;
    }
    for (uint32_t k = lane; k < 2u * n; k += 64u) dst.hot[2 * d0 + k] = src.hot[2 * s0 + k];
    if (cold)
        for (uint32_t k = lane; k < n; k += 64u) dst.cold[d0 + k] = src.cold[s0 + k];
}

__device__ inline SphRec load_sph(const SphRec *p)
{
    uint4 u = *reinterpret_cast<const uint4 *>(p);
    SphRec s;
    s.owner = u.x;
    s.rad = __uint_as_float(u.y);
    s.mat = u.z;
    s.tcomp = u.w;
    return s;
}

// Exact FP64 centre of a sphere: owner position (+ R(q) p for clump spheres).
__device__ inline void sphere_centre(const OwnerRec &r, const SphRec &s, const double *q,
                                     const float *tpos, const Origin &org, double *x)
{
    double X0 = decode_axis(r.vox, r.off[0], org.o[0], 0);
    double X1 = decode_axis(r.vox, r.off[1], org.o[1], 1);
    double X2 = decode_axis(r.vox, r.off[2], org.o[2], 2);
    if (s.tcomp == DEM_NO_COMP) {
        x[0] = X0;
        x[1] = X1;
        x[2] = X2;
        return;
    }
    const double *qq = q + 4 * (size_t)s.owner;
    double4 qv = *reinterpret_cast<const double4 *>(qq);
    Mat3d R = rot_from_q(qv.x, qv.y, qv.z, qv.w);
    float4 p = *reinterpret_cast<const float4 *>(tpos + 4 * (size_t)s.tcomp);
    double d[3];
    rot_apply(R, (double)p.x, (double)p.y, (double)p.z, d);
    x[0] = X0 + d[0];
    x[1] = X1 + d[1];
    x[2] = X2 + d[2];
}

// Bin of a coordinate along one axis: cells 1 .. n-2 hold the domain (0
// and n-1 are an empty guard layer, so a 3x3x3 stencil never leaves the
// grid); coordinates outside fall into the outermost inner cells.
__device__ inline int bin_coord(double x, double lo, double inv_b, int n)
{
    double t = floor((x - lo) * inv_b);
    int c;
    if (!(t >= 0.0)) c = 0;
    else if (t > (double)(n - 3)) c = n - 3;
    else c = (int)t;
    return c + 1;
}

// Bin key (x fastest) of a sphere centre.
__device__ inline uint32_t bin_key(const Grid &g, const double *x)
{
    const int cx = bin_coord(x[0], g.lo[0], g.inv_b, g.nx);
    const int cy = bin_coord(x[1], g.lo[1], g.inv_b, g.ny);
    const int cz = bin_coord(x[2], g.lo[2], g.inv_b, g.nz);
    return ((uint32_t)cz * (uint32_t)g.ny + (uint32_t)cy) * (uint32_t)g.nx + (uint32_t)cx;
}

// Wall w of a launch's wall table, read through the constant address space:
// the table is never written while a kernel runs, and with a uniform index
// the read is a scalar load, not one vector memory round trip per wall
// (a kernel that has stored to memory before its wall loop would otherwise
// read the table with vector loads).
__device__ inline WallDev wall_at(const WallDev *walls, int w)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) WallDev *)walls)[w];
#else
    return walls[w];   // (the host pass only parses device functions)
#endif
}

__device__ inline void wall_point(const WallDev &w, int64_t step, double h, double *p)
{
    double t = (double)step * h;
    p[0] = w.geom[0] + w.vel[0] * t;
    p[1] = w.geom[1] + w.vel[1] * t;
    p[2] = w.geom[2] + w.vel[2] * t;
}

// ---------------------------------------------------------------------------
// triangle facets of rigid meshes
// ---------------------------------------------------------------------------
// The pose of mesh g among the (at most MAX_MESHES) poses passed by value:
// selected with constant indices so the kernel arguments are never copied
// to private memory.
__device__ inline MeshPose pose_of(const MeshPoses &P, int32_t g)
{
    MeshPose r = P.m[0];
#pragma unroll
    for (int k = 1; k < MAX_MESHES; ++k)
        if (g == k) r = P.m[k];
    return r;
}

// World vertices of a facet: p + R v for each vertex v.
__device__ inline void facet_world(const TriDev &t, const MeshPose &P, double *w)
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const double x0 = t.v[3 * v], x1 = t.v[3 * v + 1], x2 = t.v[3 * v + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            w[3 * v + k] = P.p[k] + ((P.R[3 * k] * x0 + P.R[3 * k + 1] * x1) + P.R[3 * k + 2] * x2);
    }
}

__device__ inline double dot3d(const double *u, const double *v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; }

// Closest point q of the triangle (a, b, c) to p by the Voronoi-region test
// on barycentric quantities (Ericson, Real-Time Collision Detection, 2005,
// Sec. 5.1.5): a vertex, a point of an edge, or the projection onto the face.
__device__ inline void tri_closest(const double *a, const double *b, const double *c, const double *p, double *q)
{
    double e1[3], e2[3], r[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
        r[k] = p[k] - a[k];
    }
    const double s1 = dot3d(e1, r), s2 = dot3d(e2, r);
    if (s1 <= 0.0 && s2 <= 0.0) {
        for (int k = 0; k < 3; ++k) q[k] = a[k];
        return;
    }
    for (int k = 0; k < 3; ++k) r[k] = p[k] - b[k];
    const double s3 = dot3d(e1, r), s4 = dot3d(e2, r);
    if (s3 >= 0.0 && s4 <= s3) {
        for (int k = 0; k < 3; ++k) q[k] = b[k];
        return;
    }
    const double uc = s1 * s4 - s3 * s2;
    if (uc <= 0.0 && s1 >= 0.0 && s3 <= 0.0) {
        const double t = s1 / (s1 - s3);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + t * e1[k];
        return;
    }
    for (int k = 0; k < 3; ++k) r[k] = p[k] - c[k];
    const double s5 = dot3d(e1, r), s6 = dot3d(e2, r);
    if (s6 >= 0.0 && s5 <= s6) {
        for (int k = 0; k < 3; ++k) q[k] = c[k];
        return;
    }
    const double ub = s5 * s2 - s1 * s6;
    if (ub <= 0.0 && s2 >= 0.0 && s6 <= 0.0) {
        const double t = s2 / (s2 - s6);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + t * e2[k];
        return;
    }
    const double ua = s3 * s6 - s5 * s4;
    const double g43 = s4 - s3, g56 = s5 - s6;
    if (ua <= 0.0 && g43 >= 0.0 && g56 >= 0.0) {
        const double t = g43 / (g43 + g56);
        for (int k = 0; k < 3; ++k) q[k] = b[k] + t * (c[k] - b[k]);
        return;
    }
    const double inv = 1.0 / ((ua + ub) + uc);
    const double tv = ub * inv, tw = uc * inv;
    for (int k = 0; k < 3; ++k) q[k] = (a[k] + e1[k] * tv) + e2[k] * tw;
}

// Squared distance of x to the facet with world vertices w[9], and the
// closest point.
__device__ inline double facet_dist2(const double *w, const double *x, double *q)
{
    tri_closest(w, w + 3, w + 6, x, q);
    const double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
    return (dx * dx + dy * dy) + dz * dz;
}
