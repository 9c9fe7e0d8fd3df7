// Per-step dynamics for gfx950: Hertz-Mindlin contact forces, ordered
// reduction onto owners, explicit integration (paper Sec. 4.1, Eqs. (1)-(3);
// default-model walk-through of Sec. 4.2.1).
//
// k_force: one thread per sphere i walks its row of the active set (the
// contacts where i is the lower id, geometry A), in ascending partner order.
// The overlap, the normal and the contact point are evaluated in FP64
// registers from exact sphere centres; the force law runs in FP32.  The
// thread keeps the running sum of the forces and torques on A in registers
// (one 24-byte write per sphere instead of one per contact) and writes the
// reaction on B (force and torque about B's owner) per contact.  Pairs that
// do not touch (false positives of the margin) get exactly zero force and
// their history is released (reset to zero).
//
// k_fold_integrate: one thread per owner folds, for each of its spheres in
// order, the A-side sum and then the B-side reactions in ascending contact
// order -- a fixed sequential order, so adding the +0.0 terms of false
// positives changes no bit -- then integrates: semi-implicit Euler on the
// velocity (FP32 storage), FP64 position update re-encoded to voxel +
// offset, FP64 quaternion update by the exponential map for clumps.
// Single spheres keep their angular velocity in the world frame (their
// orientation has no physical effect).
//
// k_step_fused: the same step in one launch (one thread per owner, its
// B-side contacts evaluated again from their A side), the default of
// dem_step; see its comment below.
#include "dem_device.h"

#include <hip/hip_ext.h>

namespace {

constexpr int TPB = 256;

inline unsigned nblocks(int64_t n, int t = TPB)
{
    int64_t g = (n + t - 1) / t;
    return (unsigned)(g < 1 ? 1 : g);
}

// Blocks of the fused step (one per 256 owners; with fixed families at most
// FIXED_BLOCKS, each thread taking several owners).  The per-block speed
// maxima of the last step are in blkmax[0 .. step_blocks).
constexpr unsigned FIXED_BLOCKS = 2048;
inline unsigned step_blocks(const DynArgs &a)
{
    const unsigned b = nblocks(a.n_owners);
    return a.has_fixed && !a.two_kernel && b > FIXED_BLOCKS ? FIXED_BLOCKS : b;
}

struct OwnerKin {
    double X[3];     // owner centre (exact)
    float3 v;        // velocity
    float3 w;        // angular velocity in the world frame
    float mass;
};

__device__ inline void owner_kin(const OwnerRec &r, const SphRec &s, const OwnerAux *aux, const double *q,
                                 const float *tpos, const Origin &org, OwnerKin &k, double *xs)
{
    k.X[0] = decode_axis(r.vox, r.off[0], org.o[0], 0);
    k.X[1] = decode_axis(r.vox, r.off[1], org.o[1], 1);
    k.X[2] = decode_axis(r.vox, r.off[2], org.o[2], 2);
    k.v = f3(r.v[0], r.v[1], r.v[2]);
    k.mass = r.mass;
    if (s.tcomp == DEM_NO_COMP) {
        k.w = f3(r.w[0], r.w[1], r.w[2]);
        xs[0] = k.X[0];
        xs[1] = k.X[1];
        xs[2] = k.X[2];
        return;
    }
    double4 qv = *reinterpret_cast<const double4 *>(q + 4 * (size_t)s.owner);
    Mat3d R = rot_from_q(qv.x, qv.y, qv.z, qv.w);
    float4 p = *reinterpret_cast<const float4 *>(tpos + 4 * (size_t)s.tcomp);
    double d[3];
    rot_apply(R, (double)p.x, (double)p.y, (double)p.z, d);
    xs[0] = k.X[0] + d[0];
    xs[1] = k.X[1] + d[1];
    xs[2] = k.X[2] + d[2];
    double wb[3];
    rot_apply(R, (double)r.w[0], (double)r.w[1], (double)r.w[2], wb);
    k.w = f3((float)wb[0], (float)wb[1], (float)wb[2]);
}

__device__ inline bool stopped(const DevCounters *c, int64_t step)
{
    return c->stop_cd != 0u || c->div[(step + 1) & 1] != 0u;
}

// A step halted by the divergence of the step before marks itself diverged
// too, so that every later step of the call halts as well (the flags are
// kept per step parity so that no block of a step sees its own step's flag).
__device__ inline void halt_mark(DevCounters *c, int64_t step)
{
    if (c->div[(step + 1) & 1] != 0u) c->div[step & 1] = 1u;
}

__device__ inline float4 load_hist(const float *hx, const float *hy, const float *hz, const float *hw,
                                   uint32_t c, int rolling)
{
    return make_float4(hx[c], hy[c], hz[c], rolling ? hw[c] : 0.f);
}

// History arrays of a set and the contact's index in them; with `os`
// set, the arrays are those of the previous set (the step right after an
// adoption) and the pair's history is found by partner `kj` in that set's
// row of sphere `ki` (rows are sorted by partner; a pair it does not list
// starts from zero).
struct HistIn {
    const float *x, *y, *z, *w;
    uint32_t c;
    const uint32_t *os = nullptr, *oj = nullptr;
    uint32_t ki = 0, kj = 0;
};

__device__ inline float4 hist_get(const HistIn &h, int rolling)
{
    if (!h.os) return load_hist(h.x, h.y, h.z, h.w, h.c, rolling);
    const uint32_t e = h.os[h.ki + 1];
    uint32_t lo = h.os[h.ki], hi = e;
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (h.oj[mid] < h.kj) lo = mid + 1u;
        else hi = mid;
    }
    if (lo < e && h.oj[lo] == h.kj) return load_hist(h.x, h.y, h.z, h.w, lo, rolling);
    return make_float4(0.f, 0.f, 0.f, 0.f);
}

// One contact evaluated from the side of sphere A (the lower id of the pair
// or the sphere of a sphere-wall pair): overlap and normal in FP64, the
// Hertz-Mindlin law with tangential history in FP32.  `hold` is the contact's
// history before the step (read only once the pair is found touching: most
// pairs of a margin set are not); the result holds the new one.  Both the A-side
// sum and the B-side reaction of a contact are taken from this one function,
// so a contact gives the same bits wherever it is evaluated.
struct ContactOut {
    float3 F;        // force on A (normal + tangential)
    float3 Ft;       // F plus the rolling-resistance force (torques only)
    float3 armA;     // contact point minus A's owner centre
    float3 armB;     // contact point minus B's owner centre (wall: wall point; facet: mesh reference point)
    float4 h;        // history after the step (xi, contact age)
    bool touching;
    double gap;      // (GAPW) the pair's gap, exact in FP64; negative when touching
};

// Duration of a contact's first impact, during which rolling resistance is
// held back (the default model's walk-through, Sec. 4.2.1): the contact is
// taken as the linear spring-dashpot m x'' + c x' + k x = 0 with the
// walk-through's simplified constants k = (4/3) E* R_e^(1/2) and
// c = -2 sqrt((5/3) m E*) beta R_e^(1/4), R_e = sqrt(R_bar), and an impact
// lasts half a period of its damped oscillation, pi / w_d with
// w_d^2 = k / m - (c / 2m)^2.  An overdamped contact (w_d^2 <= 0) has no such
// phase: -1.
__device__ __forceinline__ float impact_time(float Estar, float beta, float Rbar, float m)
{
    const float Re = sqrtf(Rbar);
    const float k = (4.0f / 3.0f) * Estar * sqrtf(Re);
    const float c = -2.0f * sqrtf((5.0f / 3.0f) * m * Estar) * beta * sqrtf(sqrtf(Re));
    const float zeta = c / (2.0f * sqrtf(k * m));   // damping ratio (>= 0: beta <= 0)
    if (!(zeta < 1.0f)) return -1.0f;
    return 3.14159265358979f * sqrtf(m / (k * (1.0f - zeta * zeta)));
}

// Mindlin tangential spring-dashpot with the Coulomb limit (Sec. 4.1
// Eq. (2); the walk-through's form of the limit, reading R3): the trial
// force -(k_t xi + c_t u_t); above mu |F| it is scaled down to mu |F| and the
// displacement xi is set back to the value that force implies,
// xi = -(f_t + c_t u_t) / k_t; a trial force below 1e-12 N is zero.
__device__ __forceinline__ float3 tangential_force(const MatPair &mq, float sqrtRd, float m, float3 F, float3 ut,
                                                   float3 &xi)
{
    const float kt = 8.0f * mq.Gstar * sqrtRd;
    const float ct = -1.8257418583505538f * mq.beta * sqrtf(m * kt);   // 2 sqrt(5/6) |beta| sqrt(m k_t)
    const float3 ft = (-kt) * xi - ct * ut;
    const float mag = sqrtf(dot3(ft, ft));
    if (!(mag > 1e-12f)) return f3(0.f, 0.f, 0.f);
    const float limit = mq.mu * sqrtf(dot3(F, F));
    if (mag <= limit) return ft;
    const float3 fl = (limit / mag) * ft;
    xi = (-1.0f / kt) * (fl + ct * ut);
    return fl;
}

// FACETS: the set may hold sphere-facet contacts (systems with meshes; the
// FP64 closest-point code raises the register demand, so systems without
// meshes use the variant without it).
// KNOWN_B: B is a sphere whose record and kinematics the caller already
// holds (sBk, kBk, xBk; the fused step evaluates its B-list entries with
// its own sphere as B); otherwise B is loaded from jp.  SINGLES: every owner
// is one sphere, so B's owner record is at jp and is loaded with its sphere
// record rather than after it.
// GAPW: also report the pair's gap (out.gap) when it does not touch.
template <bool FACETS, bool KNOWN_B = false, bool SINGLES = false, bool GAPW = false>
__device__ __forceinline__ void contact_eval(const DynArgs &a, const SphRec &sA, const OwnerKin &kA,
                                             const double *xA, uint32_t jp, const HistIn &hin, ContactOut &out,
                                             const SphRec *sBk = nullptr, const OwnerKin *kBk = nullptr,
                                             const double *xBk = nullptr)
{
    const int64_t Ns = a.n_spheres;
    const double radA = (double)sA.rad;
    const float hf = (float)a.h;
    double nrm[3], delta = 0.0, XB[3];
    float Rbar = 0.f, mbar = 0.f;
    float3 vB = f3(0.f, 0.f, 0.f), wB = f3(0.f, 0.f, 0.f);
    uint32_t matB = 0;
    bool touching = false;
    if (KNOWN_B || (int64_t)jp < Ns) {
        SphRec sB;
        OwnerKin kB;
        double xB[3];
        if (KNOWN_B) {
            sB = *sBk;
            kB = *kBk;
            xB[0] = xBk[0];
            xB[1] = xBk[1];
            xB[2] = xBk[2];
        } else {
            // (the whole record in one round trip: reading the cold part
            // only once the pair is found touching costs touching pairs a
            // second round trip, which the step pays for more than the
            // bytes)
            sB = load_sph(a.sph + jp);
            const OwnerRec rB = load_rec(a.recs, SINGLES ? jp : sB.owner);
            owner_kin(rB, sB, a.aux, a.q, a.tpos, a.org, kB, xB);
        }
        double dx = xA[0] - xB[0], dy = xA[1] - xB[1], dz = xA[2] - xB[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        double radB = (double)sB.rad;
        double T = radA + radB;
        touching = d2 < T * T;
        if (GAPW) out.gap = touching ? -1.0 : sqrt(d2) - T;
        if (touching) {
            double d = sqrt(d2);
            nrm[0] = dx / d;
            nrm[1] = dy / d;
            nrm[2] = dz / d;
            delta = T - d;
            Rbar = (float)(radA * radB / (radA + radB));
            mbar = kA.mass * kB.mass / (kA.mass + kB.mass);
            matB = sB.mat;
            XB[0] = kB.X[0];
            XB[1] = kB.X[1];
            XB[2] = kB.X[2];
            vB = kB.v;
            wB = kB.w;
        }
    } else if (FACETS && jp >= (uint32_t)Ns + (uint32_t)a.n_walls) {
        // facet of a rigid mesh: normal from the closest point of the facet
        // to the centre; the facet acts as a flat surface (R = r_A) of
        // infinite mass moving with the mesh
        const TriDev t = a.tri[jp - (uint32_t)Ns - (uint32_t)a.n_walls];
        const MeshPose P = a.poses[t.mesh];
        double w[9], q[3];
        facet_world(t, P, w);
        const double d2 = facet_dist2(w, xA, q);
        touching = d2 < radA * radA && d2 > 0.0;
        if (GAPW) out.gap = touching || !(d2 > 0.0) ? -1.0 : sqrt(d2) - radA;
        if (touching) {
            const double d = sqrt(d2);
            nrm[0] = (xA[0] - q[0]) / d;
            nrm[1] = (xA[1] - q[1]) / d;
            nrm[2] = (xA[2] - q[2]) / d;
            delta = radA - d;
            Rbar = (float)radA;
            mbar = kA.mass;
            matB = (uint32_t)P.mat;
            XB[0] = P.p[0];
            XB[1] = P.p[1];
            XB[2] = P.p[2];
            vB = f3(P.vel[0], P.vel[1], P.vel[2]);
            wB = f3(P.omega[0], P.omega[1], P.omega[2]);
        }
    } else {
        const WallDev wd = a.walls[jp - (uint32_t)Ns];
        double p[3];
        wall_point(wd, a.step, a.h, p);
        double rx = xA[0] - p[0], ry = xA[1] - p[1], rz = xA[2] - p[2];
        if (wd.type == 0) {
            double sd = (rx * wd.geom[3] + ry * wd.geom[4]) + rz * wd.geom[5];
            touching = sd < radA;
            if (GAPW) out.gap = touching ? -1.0 : sd - radA;
            if (touching) {
                nrm[0] = wd.geom[3];
                nrm[1] = wd.geom[4];
                nrm[2] = wd.geom[5];
                delta = radA - sd;
                Rbar = (float)radA;
            }
        } else {
            double ax = (rx * wd.geom[3] + ry * wd.geom[4]) + rz * wd.geom[5];
            double hl = 0.5 * wd.geom[7];
            double px = rx - ax * wd.geom[3], py = ry - ax * wd.geom[4], pz = rz - ax * wd.geom[5];
            double d2 = (px * px + py * py) + pz * pz;
            double T = wd.geom[6] + radA;
            touching = (ax <= hl && ax >= -hl) && d2 < T * T && d2 > 0.0;
            // (apart: at least as far as the farther of the two bounds of
            // the touching region, the radius and the axial extent)
            if (GAPW) out.gap = touching ? -1.0 : fmax(sqrt(d2) - T, fabs(ax) - hl);
            if (touching) {
                double d = sqrt(d2);
                nrm[0] = px / d;
                nrm[1] = py / d;
                nrm[2] = pz / d;
                delta = T - d;
                Rbar = (float)(radA * wd.geom[6] / (radA + wd.geom[6]));
            }
        }
        if (touching) {
            mbar = kA.mass;
            matB = (uint32_t)wd.mat;
            XB[0] = p[0];
            XB[1] = p[1];
            XB[2] = p[2];
            vB = f3((float)wd.vel[0], (float)wd.vel[1], (float)wd.vel[2]);
            wB = f3((float)wd.omega[0], (float)wd.omega[1], (float)wd.omega[2]);
        }
    }
    out.touching = touching;
    if (!touching) {
        out.h = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const float4 hold = hist_get(hin, a.rolling);
    // contact point in the middle of the overlap; arms to both owner centres
    const double sc = radA - 0.5 * delta;
    double cp[3] = {xA[0] - sc * nrm[0], xA[1] - sc * nrm[1], xA[2] - sc * nrm[2]};
    const float3 armA = f3((float)(cp[0] - kA.X[0]), (float)(cp[1] - kA.X[1]), (float)(cp[2] - kA.X[2]));
    const float3 armB = f3((float)(cp[0] - XB[0]), (float)(cp[1] - XB[1]), (float)(cp[2] - XB[2]));
    const float3 n = f3((float)nrm[0], (float)nrm[1], (float)nrm[2]);
    const MatPair mq = a.mat[(size_t)sA.mat * (size_t)a.n_mat + matB];
    // relative velocity of A with respect to B at the contact point
    // (linear parts first, so their difference is exact-ish)
    const float3 rotA = cross3(kA.w, armA), rotB = cross3(wB, armB);
    const float3 u = (kA.v - vB) + (rotA - rotB);
    const float pn = dot3(u, n);
    const float3 ut = u - pn * n;
    float3 xi = f3(hold.x, hold.y, hold.z);
    xi = xi + hf * ut;
    xi = xi - dot3(xi, n) * n;
    const float df = (float)delta;
    const float sqrtRd = sqrtf(Rbar * df);
    const float Sn = 2.0f * mq.Estar * sqrtRd;
    const float kn = (2.0f / 3.0f) * Sn;
    const float c56 = 1.8257418583505538f;   // 2 sqrt(5/6)
    const float gn = c56 * mq.beta * sqrtf(Sn * mbar);
    float3 F = (kn * df + gn * pn) * n;
    // rolling resistance (Sec. 4.1 Eq. (2), Sec. 4.3.1): a torque-only force
    // of magnitude C_rr |F| along the rolling part of the relative velocity,
    // held back during the contact's first impact
    float3 Fr = f3(0.f, 0.f, 0.f);
    float age = 0.f;
    if (a.rolling) {
        age = hold.w + hf;
        if (mq.crr > 0.0f && age > impact_time(mq.Estar, mq.beta, Rbar, mbar)) {
            const float3 vr = rotB - rotA;
            const float vrn = sqrtf(dot3(vr, vr));
            if (vrn > 1e-12f) Fr = ((mq.crr * sqrtf(dot3(F, F))) / vrn) * vr;
        }
    }
    if (mq.mu > 0.0f) F = F + tangential_force(mq, sqrtRd, mbar, F, ut, xi);
    out.F = F;
    out.Ft = F + Fr;
    out.armA = armA;
    out.armB = armB;
    out.h = make_float4(xi.x, xi.y, xi.z, age);
}

__device__ inline void store_hist(float *hx, float *hy, float *hz, float *hw, uint32_t c, float4 h, int rolling)
{
    hx[c] = h.x;
    hy[c] = h.y;
    hz[c] = h.z;
    if (rolling) hw[c] = h.w;
}

// Where the fused step puts the new history of a wave's A rows.  Rows of
// consecutive owners are consecutive, so a wave's rows are one range
// [c0, c0 + n) of the set.  Its first HIST_STAGE entries are put in the
// wave's LDS slice and written out together, in whole lines, once the
// wave's owners are done (the rest go straight to memory); written per
// lane, each store would fill a few bytes of lines spread over the range
// while they wait for their other entries, and the L2 writes such lines
// back several times.
constexpr uint32_t HIST_STAGE = 512;   // entries per wave (4 components: 8 KiB)

struct HistOut {
    float *x, *y, *z, *w;
    float *lds;      // the wave's slice, component k at k * HIST_STAGE; nullptr: write to x..w directly
    uint32_t c0;     // the range's first entry
};

__device__ inline void put_hist(const HistOut &ho, uint32_t c, float4 h, int rolling)
{
    const uint32_t k = c - ho.c0;
    if (ho.lds && k < HIST_STAGE) {
        ho.lds[k] = h.x;
        ho.lds[HIST_STAGE + k] = h.y;
        ho.lds[2 * HIST_STAGE + k] = h.z;
        if (rolling) ho.lds[3 * HIST_STAGE + k] = h.w;
    } else {
        store_hist(ho.x, ho.y, ho.z, ho.w, c, h, rolling);
    }
}

// Two-kernel path (forces without integration): A-side sums per sphere and
// the reaction on B per contact, history updated in place.
template <bool FACETS>
__global__ void __launch_bounds__(TPB) k_force(DynArgs a, const uint32_t *start, const uint32_t *jarr,
                                               float *hx, float *hy, float *hz, float *hw, float *aF, float *aT,
                                               float *bF, float *bT, int64_t cap, const DevCounters *ctr)
{
    int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= a.n_spheres) return;
    if (stopped(ctr, a.step)) return;
    const int64_t Ns = a.n_spheres;
    float3 FA = f3(0.f, 0.f, 0.f), TA = f3(0.f, 0.f, 0.f);
    const uint32_t c0 = start[i], c1 = start[i + 1];
    if (c0 < c1) {
        const SphRec sA = load_sph(a.sph + i);
        const OwnerRec rA = load_rec(a.recs, sA.owner);
        OwnerKin kA;
        double xA[3];
        owner_kin(rA, sA, a.aux, a.q, a.tpos, a.org, kA, xA);
        for (uint32_t c = c0; c < c1; ++c) {
            ContactOut co;
            contact_eval<FACETS>(a, sA, kA, xA, jarr[c], HistIn{hx, hy, hz, hw, c}, co);
            store_hist(hx, hy, hz, hw, c, co.h, a.rolling);
            if (!co.touching) {
                bF[c] = 0.f;
                bF[cap + c] = 0.f;
                bF[2 * cap + c] = 0.f;
                bT[c] = 0.f;
                bT[cap + c] = 0.f;
                bT[2 * cap + c] = 0.f;
                continue;
            }
            FA = FA + co.F;
            TA = TA + cross3(co.armA, co.Ft);
            const float3 mF = f3(-co.F.x, -co.F.y, -co.F.z);
            const float3 tB = cross3(co.armB, f3(-co.Ft.x, -co.Ft.y, -co.Ft.z));
            bF[c] = mF.x;
            bF[cap + c] = mF.y;
            bF[2 * cap + c] = mF.z;
            bT[c] = tB.x;
            bT[cap + c] = tB.y;
            bT[2 * cap + c] = tB.z;
        }
        // spheres without A-side contacts write nothing: the fold reads the
        // row offsets and skips them
        aF[i] = FA.x;
        aF[Ns + i] = FA.y;
        aF[2 * Ns + i] = FA.z;
        aT[i] = TA.x;
        aT[Ns + i] = TA.y;
        aT[2 * Ns + i] = TA.z;
    }
}

// Semi-implicit Euler for one owner: velocity (FP32), angular velocity
// (world frame for single spheres, body frame for clumps, whose quaternion is
// advanced in FP64 by the exponential map and written to qout; an unrotated
// clump writes its orientation qv there unchanged), FP64 position
// re-encoded on the 2^-38 m grid.  Flags divergence; returns |v|^2.
__device__ __forceinline__ float advance(const DynArgs &a, OwnerRec &r, const float *inv, bool rotating, float3 F,
                                         float3 T, const double4 qv, double *qout, DevCounters *ctr)
{
    const float hf = (float)a.h;
    const float m = r.mass;
    float3 v = f3(r.v[0], r.v[1], r.v[2]);
    v = v + hf * f3(F.x / m + a.g[0], F.y / m + a.g[1], F.z / m + a.g[2]);
    float3 w = f3(r.w[0], r.w[1], r.w[2]);
    if (!rotating) {
        w = w + hf * f3(T.x * inv[0], T.y * inv[1], T.z * inv[2]);
    } else {
        Mat3d R = rot_from_q(qv.x, qv.y, qv.z, qv.w);
        // torque into the body frame: R^T T
        const float tbx = (float)((R.m[0] * (double)T.x + R.m[3] * (double)T.y) + R.m[6] * (double)T.z);
        const float tby = (float)((R.m[1] * (double)T.x + R.m[4] * (double)T.y) + R.m[7] * (double)T.z);
        const float tbz = (float)((R.m[2] * (double)T.x + R.m[5] * (double)T.y) + R.m[8] * (double)T.z);
        w = w + hf * f3(tbx * inv[0], tby * inv[1], tbz * inv[2]);
        // q <- normalize(q (x) exp(h w / 2)) in FP64
        const double th0 = a.h * (double)w.x, th1 = a.h * (double)w.y, th2 = a.h * (double)w.z;
        const double ang = sqrt((th0 * th0 + th1 * th1) + th2 * th2);
        if (ang > 0.0) {
            // sin(x)/x and cos(x) of the half angle x; a step turns a clump by
            // far less than 0.02 rad, where their Taylor series cut after the
            // x^6 and x^8 terms are exact to below 2^-60 relative
            const double x = 0.5 * ang, x2 = x * x;
            double sinc, ch;
            if (x < 1e-2) {
                sinc = 1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0)));
                ch = 1.0 - x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0))));
            } else {
                sinc = sin(x) / x;
                ch = cos(x);
            }
            const double sh = 0.5 * sinc;   // sin(ang / 2) / ang
            const double b0 = ch, b1q = sh * th0, b2 = sh * th1, b3 = sh * th2;
            double n0 = qv.x * b0 - qv.y * b1q - qv.z * b2 - qv.w * b3;
            double n1 = qv.x * b1q + qv.y * b0 + qv.z * b3 - qv.w * b2;
            double n2 = qv.x * b2 - qv.y * b3 + qv.z * b0 + qv.w * b1q;
            double n3 = qv.x * b3 + qv.y * b2 - qv.z * b1q + qv.w * b0;
            const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2 + n3 * n3);
            *reinterpret_cast<double4 *>(qout) = make_double4(n0 / nn, n1 / nn, n2 / nn, n3 / nn);
        } else if (qout) {
            *reinterpret_cast<double4 *>(qout) = qv;
        }
    }
    // position: FP64 update, re-encoded on the 2^-38 m grid
    uint32_t iv[3];
    for (int k = 0; k < 3; ++k) {
        const float vk = k == 0 ? v.x : (k == 1 ? v.y : v.z);
        const double X = decode_axis(r.vox, r.off[k], a.org.o[k], k) + a.h * (double)vk;
        encode_axis(X, a.org.o[k], &iv[k], &r.off[k]);
    }
    r.vox = pack_vox(iv[0], iv[1], iv[2]);
    r.v[0] = v.x;
    r.v[1] = v.y;
    r.v[2] = v.z;
    r.w[0] = w.x;
    r.w[1] = w.y;
    r.w[2] = w.z;
    const float v2 = dot3(v, v);
    if (!(v2 == v2) || (a.v_err2 > 0.0f && v2 > a.v_err2) || !(dot3(w, w) == dot3(w, w)))
        ctr->div[a.step & 1] = 1u;
    return v2;
}

// Block-wide max of |v|^2 written to the block's slot (no atomics); the
// maximum over blocks is reduced only when it is read.  Returns it in
// thread 0.
__device__ __forceinline__ float block_max_v2(float v2, float *slot)
{
    __shared__ float wmax[TPB / 64];
    if (!(v2 == v2)) v2 = 3.0e38f;
    for (int d = 32; d > 0; d >>= 1) v2 = fmaxf(v2, __shfl_xor(v2, d, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v2;
    __syncthreads();
    float m = 0.0f;
    if (threadIdx.x == 0) {
        m = wmax[0];
        for (int k = 1; k < TPB / 64; ++k) m = fmaxf(m, wmax[k]);
        *slot = m;
    }
    return m;
}

// SINGLES: every owner is one sphere (sphere index == owner index), so the
// owner's sphere range and template are not read and the inverse moment of
// inertia is one isotropic value.  The owner state is loaded before the sums
// so its latency overlaps theirs.
template <bool SINGLES>
__global__ void __launch_bounds__(TPB) k_fold_integrate(DynArgs a, const uint32_t *start,
                                                        const uint32_t *bstart,
                                                        const uint32_t *bidx, const float *aF,
                                                        const float *aT, const float *bF,
                                                        const float *bT, int64_t cap, float *Fo,
                                                        float *To, int integrate, const uint8_t *oany,
                                                        DevCounters *ctr)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (stopped(ctr, a.step)) {
        if (integrate && o == 0) halt_mark(ctr, a.step);
        return;
    }
    const int64_t Ns = a.n_spheres, No = a.n_owners;
    const bool valid = o < No;
    float v2 = 0.0f;
    if (integrate && o == 0) {
        ctr->last_step_done = a.step + 1;
        ctr->contact_steps += ctr->n_contacts[a.cur];
        a.blkmax[gridDim.x] = 0.0f;   // (the slot of the split step's second kernel)
    }
    if (valid) {
        OwnerRec r;
        float inv[3];
        int32_t tmpl = -1;
        if (integrate) {
            r = load_rec(a.recs, o);
            if (SINGLES) {
                inv[0] = inv[1] = inv[2] = a.inv_i[o];
            } else {
                const OwnerAux ax = a.aux[o];
                inv[0] = ax.inv_moi[0];
                inv[1] = ax.inv_moi[1];
                inv[2] = ax.inv_moi[2];
                tmpl = ax.tmpl;
            }
        }
        float3 F = f3(0.f, 0.f, 0.f), T = f3(0.f, 0.f, 0.f);
        const uint32_t s0 = SINGLES ? (uint32_t)o : a.own_sph0[o];
        const uint32_t s1 = SINGLES ? (uint32_t)o + 1u : a.own_sph0[o + 1];
        for (uint32_t s = s0; s < s1; ++s) {
            if (start[s] != start[s + 1]) {
                F = F + f3(aF[s], aF[Ns + s], aF[2 * Ns + s]);
                T = T + f3(aT[s], aT[Ns + s], aT[2 * Ns + s]);
            }
            const uint32_t b1 = bstart[s + 1];
            for (uint32_t b = bstart[s]; b < b1; ++b) {
                const uint32_t c = bidx[b];
                F = F + f3(bF[c], bF[cap + c], bF[2 * cap + c]);
                T = T + f3(bT[c], bT[cap + c], bT[2 * cap + c]);
            }
        }
        if (!integrate) {
            Fo[o] = F.x;
            Fo[No + o] = F.y;
            Fo[2 * No + o] = F.z;
            To[o] = T.x;
            To[No + o] = T.y;
            To[2 * No + o] = T.z;
        } else if (!(a.has_fixed && (oany[o] & 2u))) {
            // orientation updated in place (owners of fixed families keep their state)
            const bool rot = !SINGLES && tmpl >= 0;
            double *qp = a.q + 4 * (size_t)o;
            const double4 qv = rot ? *reinterpret_cast<const double4 *>(qp) : make_double4(1.0, 0.0, 0.0, 0.0);
            v2 = advance(a, r, inv, rot, F, T, qv, rot ? qp : nullptr, ctr);
            store_rec(a.recs, o, r);
        }
    }
    if (integrate) block_max_v2(v2, a.blkmax + blockIdx.x);
}

// One whole step per owner.  Its spheres' A rows are evaluated (history
// written to the second buffer); each B-list entry is evaluated again from
// its A sphere with the same function (reading the history before the step),
// so the owner needs no reaction written by another thread.  The sums run in
// the order of the two-kernel path -- per sphere the A-row sum, then the
// B-side reactions by ascending contact index -- and the integration is the
// same, so both paths give the same bits.  Reads (a.recs, a.q, history),
// writes (rec_out, q_out, second history): no thread reads what another
// writes.  When the step is stopped (capacity or divergence) the state and
// history are copied unchanged.  SINGLES: every owner is one sphere; FACETS:
// the set may hold sphere-facet contacts; FIXED: some owner is in a fixed
// family; STAGE: the history of a wave's rows goes through LDS (sets with
// many contacts per sphere; with few, looking up each wave's range costs
// more than it saves); REMAP: the first step on a newly adopted set, which
// reads the old history from the previous set (DynArgs::rm_*); WO: a step
// that also does a work order's first binning step (DynArgs::wo_*).
// Systems with clumps or meshes get 3 waves per SIMD: the clump rotation
// and the FP64 closest point would otherwise spill registers to scratch
// inside the contact loop, which costs more than the lost occupancy.

// What the contact part of an owner's step hands to its integration.
struct OwnerStep {
    OwnerRec r;
    float inv[3];
    int32_t tmpl;
    double4 qv;
    float3 F, T;
    bool advance;    // the owner is integrated (not in a fixed family)
};

// Pairs proven apart (see DynArgs::gap).  Per step, room for the rounding
// of two re-encoded positions (2^-38 m per axis each) and of the facet and
// wall poses; per pair, room for the rounding of its FP64 gap and of the
// touching test.  Both are far above those roundings and far below any gap
// worth skipping.
constexpr double GAP_STEP_SLACK = 1e-10;
constexpr double GAP_PAIR_SLACK = 1e-9;
constexpr int GAP_SLOTS = 64;    // speed slots per step
constexpr int GAP_STRIDE = 16;   // floats from one slot to the next (64 B)

__device__ inline float *gap_slot(const DynArgs &a, int64_t step, uint32_t k)
{
    return a.gvs + ((size_t)(step % 3) * GAP_SLOTS + (k & (GAP_SLOTS - 1))) * GAP_STRIDE;
}

// The reach D of this step (every lane of the wave calls it; all waves of
// the launch get the same value): 0 on the first step of a chain, else the
// previous step's reach plus how far any two surfaces can have closed in
// during that step: h times twice the largest sphere speed it integrated
// (its blocks' maxima, in the speed slots) plus the fastest wall or mesh
// point, plus the slack.
__device__ inline double gap_reach(const DynArgs &a)
{
    if (a.gap != 2) return 0.0;
    const uint32_t lane = threadIdx.x & 63u;
    float m = *gap_slot(a, a.step + 2, lane);
    for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
    // (the maxima are FP32 squares: a relative allowance of 1e-6 on the speed)
    const double v = sqrt((double)m) * (1.0 + 1e-6);
    return a.gD[(a.step + 1) & 1] + a.h * (2.0 * v + a.vgeom) + GAP_STEP_SLACK;
}

// The speed bound of an integrated owner for the reach: |v| + |w| arm
// (arm 0 for single spheres), squared, with a relative allowance of 1e-6
// for its FP32 rounding.
__device__ inline float reach_speed2(const OwnerRec &r, float arm)
{
    const float v = sqrtf((r.v[0] * r.v[0] + r.v[1] * r.v[1]) + r.v[2] * r.v[2]);
    const float w = sqrtf((r.w[0] * r.w[0] + r.w[1] * r.w[1]) + r.w[2] * r.w[2]);
    const float sp = (v + w * arm) * 1.000001f;
    return sp * sp;
}

// The key of a pair evaluated at reach D with gap g: (g - slack) + D
// rounded down to FP32; a pair that touches or nearly does gets a key no
// reach can pass.
__device__ inline float gap_key(double g, double D)
{
    if (!(g > GAP_PAIR_SLACK)) return -3.0e38f;
    const double k = (g - GAP_PAIR_SLACK) + D;
    float f = (float)k;
    if ((double)f > k) f = __uint_as_float(__float_as_uint(f) - 1u);   // (k > 0: one ulp down)
    return f;
}

// The contact part of one owner's step (see k_step_fused): the sums F, T of
// the forces and torques on it, its rows' new history put through ho.
// GAP (single spheres without fixed families, dense sets): items are
// skipped by the pairs' keys and the A rows' keys written (DynArgs::gap; Dn
// is the step's reach), and an item's indices are loaded two items ahead,
// its key one item ahead.
// BOUNDS (clumps, the owners of a set's list of owners with contacts): the
// first sphere and the row and B-list bounds of the owner's spheres come
// with its record in the list (lrec, AcsBuf::olist), so that neither they
// nor a sphere without items cost a round trip of their own (an owner
// whose record holds no lengths loads them per sphere); the owner's flag is
// known (it has contacts, and such runs have no fixed families) and is not
// read.
struct ListRec {
    uint4 h, c;
};

template <bool SINGLES, bool FACETS, bool FIXED, bool AHEAD, bool REMAP, bool GAP = false, bool BOUNDS = false>
__device__ __forceinline__ void owner_forces(const DynArgs &a, const int64_t o, const uint32_t *start,
    const uint32_t *jarr, const uint32_t *bstart, const uint32_t *bidx, const uint32_t *bsrc, const uint8_t *oany,
    const uint8_t fl_fixed, const float *hx, const float *hy, const float *hz, const float *hw, const HistOut &ho,
    OwnerStep &st, const OwnerRec *pre = nullptr, const double Dn = 0.0, const ListRec lrec = ListRec{})
{
    static_assert(!GAP || !FIXED, "pair skipping is for systems without fixed families");
    static_assert(!BOUNDS || !FIXED, "listed owners run without fixed families");
    st.advance = false;
    // The owner's flag byte, written with the set (bit 0: the owner has a
    // contact in it; bit 1: the owner is in a fixed family), read by the
    // caller when FIXED (fl_fixed).  Owners of fixed families keep their
    // state, which both state buffers hold: without contacts there is
    // nothing to do; with contacts only their A rows are evaluated, for the
    // history
    if (!FIXED || (fl_fixed & 3u) != 2u) {
        // every per-owner load is issued here, none waits for another: the
        // record, the inertia, the orientation (clump systems) and (without
        // fixed families) the flag
        OwnerRec &r = st.r;
        r = pre ? *pre : load_rec(a.recs, o);
        st.tmpl = -1;
        st.qv = make_double4(1.0, 0.0, 0.0, 0.0);
        if (SINGLES) {
            st.inv[0] = st.inv[1] = st.inv[2] = a.inv_i[o];
        } else {
            const OwnerAux ax = a.aux[o];
            st.inv[0] = ax.inv_moi[0];
            st.inv[1] = ax.inv_moi[1];
            st.inv[2] = ax.inv_moi[2];
            st.tmpl = ax.tmpl;
            st.qv = *reinterpret_cast<const double4 *>(a.q + 4 * (size_t)o);
        }
        const uint8_t fl = FIXED ? fl_fixed : (BOUNDS ? (uint8_t)1u : oany[o]);
        const bool any = (fl & 1u) != 0;
        const bool fixed = FIXED && (fl & 2u) != 0;
        float3 F = f3(0.f, 0.f, 0.f), T = f3(0.f, 0.f, 0.f);
        const bool packed = BOUNDS && lrec.c.w != LIST_NOPACK;
        const uint32_t s0 = BOUNDS ? lrec.h.y : SINGLES ? (uint32_t)o : (any ? a.own_sph0[o] : 0u);
        const uint32_t s1 = packed ? s0 + lrec.c.w
                                   : SINGLES ? (uint32_t)o + 1u : (any ? a.own_sph0[o + 1] : 0u);
        // (packed: the next sphere's row and B-list starts, and the lengths
        // still to come, a byte per sphere)
        uint32_t pc = 0u, pb = 0u;
        uint64_t prow = 0u, pbl = 0u;
        if constexpr (BOUNDS) {
            pc = lrec.h.z;
            pb = lrec.h.w;
            prow = (uint64_t)lrec.c.x | (uint64_t)(lrec.c.y & 0xffffu) << 32;
            pbl = (uint64_t)(lrec.c.y >> 16) | (uint64_t)lrec.c.z << 16;
        }
        for (uint32_t s = s0; any && s < s1; ++s) {
            uint32_t c0, na, b0, nall;
            if (packed) {
                const uint32_t nb = (uint32_t)pbl & 0xffu;
                na = (uint32_t)prow & 0xffu;
                c0 = pc;
                b0 = pb;
                prow >>= 8;
                pbl >>= 8;
                pc += na;
                pb += nb;
                nall = na + nb;
                if (nall == 0) continue;
            } else {
                c0 = start[s];
                na = start[s + 1] - c0;
                b0 = bstart[s];
                nall = fixed ? na : na + (bstart[s + 1] - b0);
            }
            // single spheres: the sphere's own record and kinematics come
            // from the owner record already loaded, once, as geometry A of
            // its row and geometry B of its B list (for clumps, whose
            // kinematics hold more registers, they are loaded per item)
            SphRec sS{};
            OwnerKin kS{};
            double xS[3] = {0.0, 0.0, 0.0};
            if constexpr (SINGLES) {
                sS = load_sph(a.sph + s);
                owner_kin(r, sS, a.aux, a.q, a.tpos, a.org, kS, xS);
            }
            // one loop over the sphere's A row, then its B list: each item is
            // evaluated from its A side by the same function.  An item's
            // indices (contact index; partner on the A side, source sphere on
            // the B side) are loaded one item ahead (AHEAD), so that an item
            // waits for one round trip to memory (its other sphere's records),
            // not two; the variant for sparse sets of single spheres, whose
            // registers are at the limit of 4 waves per SIMD, loads them when
            // it reaches the item.
            float3 FA = f3(0.f, 0.f, 0.f), TA = f3(0.f, 0.f, 0.f);
            // the history of contact c (pair of spheres ki < kj, or sphere ki
            // and wall / facet key kj); right after an adoption, looked up
            // in the previous set
            auto hin = [&](uint32_t c, uint32_t ki, uint32_t kj) {
                HistIn h{hx, hy, hz, hw, c};
                if (REMAP) {
                    h.x = a.rm_hx;
                    h.y = a.rm_hy;
                    h.z = a.rm_hz;
                    h.w = a.rm_hw;
                    h.os = a.rm_start;
                    h.oj = a.rm_j;
                    h.ki = ki;
                    h.kj = kj;
                }
                return h;
            };
            auto fetch = [&](uint32_t t, uint32_t &cc, uint32_t &jj) {
                if (t < na) {
                    cc = c0 + t;
                    jj = jarr[cc];
                } else {
                    const uint32_t b = b0 + (t - na);
                    cc = bidx[b];
                    jj = bsrc[b];
                }
            };
            // item t (contact c, partner or source jt), its sums; skipped:
            // what a pair that does not touch gives
            auto item = [&](uint32_t t, uint32_t c, uint32_t jt, bool skip) {
                const bool aside = t < na;
                ContactOut co;
                co.touching = false;
                co.h = make_float4(0.f, 0.f, 0.f, 0.f);
                if (!skip) {
                    if constexpr (SINGLES) {
                        if (aside) {
                            contact_eval<FACETS, false, true, GAP>(a, sS, kS, xS, jt, hin(c, s, jt), co);
                            if (GAP && a.gap != 0) a.gk[c] = gap_key(co.gap, Dn);
                        } else {
                            const uint32_t iA = jt;
                            // (owner index == sphere index: both loads at once)
                            const SphRec sA = load_sph(a.sph + iA);
                            const OwnerRec rA = load_rec(a.recs, iA);
                            OwnerKin kA;
                            double xA[3];
                            owner_kin(rA, sA, a.aux, a.q, a.tpos, a.org, kA, xA);
                            contact_eval<false, true>(a, sA, kA, xA, s, hin(c, iA, s), co, &sS, &kS, xS);
                        }
                    } else {
                        const uint32_t iA = aside ? s : jt, jp = aside ? jt : s;
                        const SphRec sA = load_sph(a.sph + iA);
                        const OwnerRec rA = load_rec(a.recs, sA.owner);
                        OwnerKin kA;
                        double xA[3];
                        owner_kin(rA, sA, a.aux, a.q, a.tpos, a.org, kA, xA);
                        contact_eval<FACETS, false, false, GAP>(a, sA, kA, xA, jp, hin(c, iA, jp), co);
                        if (GAP && aside && a.gap != 0) a.gk[c] = gap_key(co.gap, Dn);
                    }
                }
                if (aside) {
                    put_hist(ho, c, co.h, a.rolling);
                    if (co.touching) {
                        FA = FA + co.F;
                        TA = TA + cross3(co.armA, co.Ft);
                    }
                    if (t + 1 == na) {
                        F = F + FA;
                        T = T + TA;
                    }
                } else {
                    float3 mF = f3(0.f, 0.f, 0.f), tB = f3(0.f, 0.f, 0.f);
                    if (co.touching) {
                        mF = f3(-co.F.x, -co.F.y, -co.F.z);
                        tB = cross3(co.armB, f3(-co.Ft.x, -co.Ft.y, -co.Ft.z));
                    }
                    F = F + mF;
                    T = T + tB;
                }
            };
            if constexpr (GAP) {
                // a skipped item waits for nothing: its key was loaded an
                // item earlier, after its indices had arrived
                const bool skipping = a.gap == 2;
                uint32_t c1 = 0, j1 = 0, c2 = 0, j2 = 0;
                float k1 = -3.0e38f;
                if (nall > 0) fetch(0, c1, j1);
                if (nall > 1) fetch(1, c2, j2);
                if (skipping && nall > 0) k1 = a.gk[c1];
                for (uint32_t t = 0; t < nall; ++t) {
                    const uint32_t c = c1, jt = j1;
                    const float key = k1;
                    c1 = c2;
                    j1 = j2;
                    if (skipping && t + 1 < nall) k1 = a.gk[c1];
                    if (t + 2 < nall) fetch(t + 2, c2, j2);
                    item(t, c, jt, skipping && (double)key - Dn > 0.0);
                }
            } else {
                uint32_t nj = 0, nc = 0;
                if (AHEAD && nall > 0) fetch(0, nc, nj);
                for (uint32_t t = 0; t < nall; ++t) {
                    if (!AHEAD) fetch(t, nc, nj);
                    const uint32_t c = nc, jt = nj;
                    if (AHEAD && t + 1 < nall) fetch(t + 1, nc, nj);
                    item(t, c, jt, false);
                }
            }
        }
        st.F = F;
        st.T = T;
        st.advance = !fixed;
    }
}

// The integration part of an owner's step; returns its |v|^2.
template <bool SINGLES>
__device__ __forceinline__ float owner_advance(const DynArgs &a, const int64_t o, OwnerStep &st, RecBuf rec_out,
                                               double *q_out, DevCounters *ctr)
{
    const bool rotating = !SINGLES && st.tmpl >= 0;
    double *qo = q_out + 4 * (size_t)o;
    // (a single sphere's orientation never changes and both buffers hold
    // it, so nothing is copied for it)
    const float v2 = advance(a, st.r, st.inv, rotating, st.F, st.T, st.qv, qo, ctr);
    store_rec(rec_out, o, st.r);
    return v2;
}

// A stopped step: the owner's state and history are copied unchanged.
template <bool SINGLES>
__device__ __forceinline__ void halt_owner(const DynArgs &a, const int64_t o, RecBuf rec_out, double *q_out, const uint32_t *start,
    const uint32_t *jarr, const uint32_t *bstart, const uint32_t *bidx, const uint32_t *bsrc, const uint8_t *oany,
    const float *hx, const float *hy, const float *hz, const float *hw, float *ox, float *oy, float *oz, float *ow,
    int64_t cap, DevCounters *ctr)
{
        store_rec(rec_out, o, load_rec(a.recs, o));
        if (!SINGLES)
            *reinterpret_cast<double4 *>(q_out + 4 * (size_t)o) =
                *reinterpret_cast<const double4 *>(a.q + 4 * (size_t)o);
        // (a set that overflowed its capacity has no valid rows to copy)
        const uint32_t s0 = SINGLES ? (uint32_t)o : a.own_sph0[o];
        const uint32_t s1 = SINGLES ? (uint32_t)o + 1u : a.own_sph0[o + 1];
        if ((int64_t)start[a.n_spheres] <= cap) {
            for (uint32_t s = s0; s < s1; ++s)
                for (uint32_t c = start[s]; c < start[s + 1]; ++c) {
                    HistIn h{hx, hy, hz, hw, c};
                    if (a.rm_start) {
                        // (right after an adoption: the history carried over
                        // from the previous set, as k_remap would have)
                        h = HistIn{a.rm_hx, a.rm_hy, a.rm_hz, a.rm_hw, c, a.rm_start, a.rm_j, s, jarr[c]};
                    }
                    store_hist(ox, oy, oz, ow, c, hist_get(h, a.rolling), a.rolling);
                }
        }
}

// The work order's first binning step for owner o (= sphere o in single-
// sphere runs) from the state r the step reads: bin key, candidate record,
// and the bin counts with the sphere's slot among its bin's spheres (one
// claim per run of equal keys in the wave, so every lane of the wave calls
// it).  The arithmetic of k_cd_prepare.
__device__ __forceinline__ void wo_front(const DynArgs &a, const int64_t o, const bool valid, const OwnerRec &r,
                                         const SphRec &sp)
{
    uint32_t key = a.wo_grid.nbins;
    double x[3] = {0.0, 0.0, 0.0};
    if (valid) {
        sphere_centre(r, sp, a.q, a.tpos, a.org, x);
        key = bin_key(a.wo_grid, x);
    }
    const uint32_t rank = wave_run_claim(a.wo_count, key, valid);
    if (valid) {
        a.wo_keys[o] = key;
        a.wo_rank[o] = rank;
        Cand c;
        c.x = x[0];
        c.y = x[1];
        c.z = x[2];
        c.r = sp.rad;
        c.id = (uint32_t)o;
        a.wo_cand[o] = c;
    }
}

// The step of the (up to) 64 consecutive owners from ow of one wave (runs
// without fixed families); every
// lane of the wave takes part (the history range is written out by all of
// them, before the owner records, so that the wait for the range's bounds
// is not a wait for those stores).  Returns the lane's |v|^2.
template <bool SINGLES, bool FACETS, bool FIXED, bool STAGE, bool REMAP, bool WO>
__device__ __forceinline__ float step_wave(const DynArgs &a, const int64_t ow, uint4 *lrec, float *lds, RecBuf rec_out, double *q_out,
    const uint32_t *start, const uint32_t *jarr, const uint32_t *bstart, const uint32_t *bidx, const uint32_t *bsrc,
    const uint8_t *oany, const float *hx, const float *hy, const float *hz, const float *hw, float *ox, float *oy,
    float *oz, float *ohw, int64_t cap, DevCounters *ctr)
{
    const int64_t No = a.n_owners;
    const uint32_t lane = threadIdx.x & 63u;
    const int64_t o = ow + lane;
    const bool valid = o < No;
    SphRec spw{};
    if (WO && valid) spw = load_sph(a.sph + o);
    // Single-sphere runs: the wave's owner records (one 3 KiB tile) move
    // through LDS in three contiguous 1 KiB loads and stores: a lane's own
    // record read as three 16-byte pieces would touch every line of the
    // tile several times.  (With STAGE the
    // slice is shared with the history staging, which is used only while
    // the records sit in registers.)  Clump runs load the record with the
    // owner's other data (inertia, orientation), which would otherwise wait
    // for it.
    const uint32_t nv = (uint32_t)(No - ow < 64 ? No - ow : 64);
    OwnerRec rpre{};
    if constexpr (SINGLES) {
        rec_copy(rec_lds(lrec, a.recs), 0, a.recs, ow, nv, lane, true);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid) rpre = load_rec(rec_lds(lrec, a.recs), lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the range of the wave's rows, read here and used only once the rows
    // are evaluated (its loads overlap the owners')
    HistOut ho{ox, oy, oz, ohw, nullptr, 0u};
    uint32_t c_end = 0;
    if constexpr (STAGE) {
        const int64_t oe = ow + 64 < No ? ow + 64 : No;
        const uint32_t sb = SINGLES ? (uint32_t)ow : a.own_sph0[ow];
        const uint32_t se = SINGLES ? (uint32_t)oe : a.own_sph0[oe];
        ho.lds = lds;
        ho.c0 = start[sb];
        c_end = start[se];
    }
    // pair skipping: the step's reach; the launch's first wave records it
    // and clears the speed slots the next step fills
    constexpr bool GAP = SINGLES && !FIXED && STAGE;
    double Dn = 0.0;
    if constexpr (GAP) {
        Dn = gap_reach(a);
        if (a.gap != 0 && ow == 0) {
            if (lane == 0) a.gD[a.step & 1] = Dn;
            *gap_slot(a, a.step + 1, lane) = 0.0f;
        }
    }
    OwnerStep st;
    st.advance = false;
    if (valid)
        owner_forces<SINGLES, FACETS, FIXED, STAGE || FACETS || !SINGLES, REMAP, GAP>(a, o, start, jarr, bstart, bidx, bsrc, oany, 0, hx, hy, hz, hw, ho, st,
                                                                                       SINGLES ? &rpre : nullptr, Dn);
    // (st.r is still the state read, before this step's update)
    if constexpr (WO) wo_front(a, o, valid, st.r, spw);
    const uint32_t n = c_end - ho.c0 < HIST_STAGE ? c_end - ho.c0 : HIST_STAGE;
    if (STAGE && n > 0) {
        // every staged entry was put by some lane of this wave.  The LDS
        // operations of a wave are performed in the order it issues them,
        // so wavefront-scope ordering is enough.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t wc0 = ho.c0;
        for (uint32_t k = lane; k < n; k += 64u) {
            ox[wc0 + k] = lds[k];
            oy[wc0 + k] = lds[HIST_STAGE + k];
            oz[wc0 + k] = lds[2 * HIST_STAGE + k];
            if (a.rolling) ohw[wc0 + k] = lds[3 * HIST_STAGE + k];
        }
    }
    if constexpr (!SINGLES) return st.advance ? owner_advance<SINGLES>(a, o, st, rec_out, q_out, ctr) : 0.0f;
    // the new records, through LDS again (after every lane is done with the
    // slice's history entries)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float v2 = 0.0f;
    if (st.advance) {
        v2 = advance(a, st.r, st.inv, false, st.F, st.T, st.qv, q_out + 4 * (size_t)o, ctr);
        store_rec(rec_lds(lrec, a.recs), lane, st.r);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    rec_copy(rec_out, ow, rec_lds(lrec, rec_out), 0, nv, lane, true);
    return v2;
}

template <bool SINGLES, bool FACETS, bool FIXED, bool STAGE, bool REMAP, bool WO>
__global__ void __launch_bounds__(TPB, (FACETS || !SINGLES) ? 3 : 4) k_step_fused(DynArgs a, RecBuf rec_out, double *q_out,
                                                    const uint32_t *start, const uint32_t *jarr,
                                                    const uint32_t *bstart, const uint32_t *bidx,
                                                    const uint32_t *bsrc, const uint8_t *oany,
                                                    const float *hx, const float *hy, const float *hz,
                                                    const float *hw, float *ox, float *oy, float *oz, float *ow,
                                                    int64_t cap, DevCounters *ctr)
{
    static_assert(!(FIXED && STAGE), "runs with fixed families do not stage");
    static_assert(!WO || (SINGLES && !FIXED && !REMAP), "work orders ride on single-sphere steps only");
    // per wave: the staged history (STAGE) and the owner records, one slice
    __shared__ uint4 wbuf[FIXED ? 1 : TPB / 64][FIXED ? 1 : (STAGE ? HIST_STAGE : 192)];
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t o0 = (int64_t)lb * blockDim.x + threadIdx.x;
    const int64_t No = a.n_owners;
    // with fixed families most owners may be dormant: each thread then takes
    // every (grid size)-th owner, so dormant owners cost their flag byte and
    // not a thread each
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // right after an adoption, an overflowed new set stops the run (every
    // block reads the same flag, so all of them halt)
    const bool rm_over = REMAP && ctr->overflow[a.rm_newbuf] != 0u;
    if (rm_over && o0 == 0) ctr->stop_cd = 1u;
    if (rm_over || stopped(ctr, a.step)) {
        if (o0 == 0) halt_mark(ctr, a.step);
        if constexpr (WO) {
            // the work order's binning is still written (from the state
            // carried over unchanged), so the detection chain reads a
            // consistent snapshot
            const bool v = o0 < No;
            OwnerRec r{};
            SphRec sp{};
            if (v) {
                r = load_rec(a.recs, o0);
                sp = load_sph(a.sph + o0);
            }
            wo_front(a, o0, v, r, sp);
        }
        if constexpr (FIXED) {
            for (int64_t o = o0; o < No; o += stride) halt_owner<SINGLES>(a, o, rec_out, q_out, start, jarr, bstart, bidx, bsrc, oany, hx, hy, hz, hw, ox, oy, oz, ow, cap, ctr);
        } else if (o0 < No) {
            const int64_t o = o0;
            halt_owner<SINGLES>(a, o, rec_out, q_out, start, jarr, bstart, bidx, bsrc, oany, hx, hy, hz, hw, ox, oy, oz, ow, cap, ctr);
        }
        return;
    }
    if (o0 == 0) {
        ctr->last_step_done = a.step + 1;
        ctr->contact_steps += ctr->n_contacts[a.cur];
        a.blkmax[gridDim.x] = 0.0f;   // (the slot of the split step's second kernel)
    }
    float v2 = 0.0f;
    // the wave's index in the block, as a wave-uniform (scalar) value
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    uint4 *lrec = FIXED ? nullptr : wbuf[wv];
    float *lds = STAGE ? reinterpret_cast<float *>(wbuf[wv]) : nullptr;
    const int64_t w0 = (int64_t)lb * blockDim.x + 64 * wv;
    if constexpr (FIXED) {
        // (no staging: the owners of a thread are not those of one wave)
        const HistOut ho{ox, oy, oz, ow, nullptr, 0u};
        for (int64_t o = o0; o < No; o += stride) {
            OwnerStep st;
            owner_forces<SINGLES, FACETS, FIXED, STAGE || FACETS || !SINGLES, REMAP>(a, o, start, jarr, bstart, bidx, bsrc, oany, oany[o], hx, hy, hz,
                                                 hw, ho, st);
            if (st.advance) v2 = fmaxf(v2, owner_advance<SINGLES>(a, o, st, rec_out, q_out, ctr));
        }
    } else if (w0 < No) {
        v2 = step_wave<SINGLES, FACETS, FIXED, STAGE, REMAP, WO>(a, w0, lrec, lds, rec_out, q_out, start, jarr, bstart, bidx, bsrc, oany, hx, hy, hz, hw, ox, oy, oz, ow, cap, ctr);
    }
    const float bm = block_max_v2(v2, a.blkmax + lb);
    // pair skipping: the block's maximum into one of the step's speed slots
    // (non-negative floats order as their bits)
    if constexpr (SINGLES && !FIXED && STAGE) {
        if (a.gap != 0 && threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned *>(gap_slot(a, a.step, lb)), __float_as_uint(bm));
    }
}


// The step of a clump system (no fixed families) whose set has few
// contacts, as two kernels.  Most owners then have no contact: for them the
// step is a stream of loads, the integration under gravity alone and
// stores, and the one-kernel step runs them at the occupancy its contact
// path allows (3 waves per SIMD).  k_step_free streams every owner at the
// occupancy of that stream: an owner whose flag says it has no contact in
// the set (bit 0 clear) is integrated with zero force and torque, exactly
// as the one-kernel step does; the others are copied and left to
// k_step_listed, which runs after it on the same stream over the set's list
// of owners with contacts and does for each what the one-kernel step does
// (owner_forces, then the integration), so both forms give the same bits.
// Each lane loads its owner's hot part (consecutive lanes, consecutive
// 32-byte parts: clump systems split their records), with the flag; the
// new hot parts go out through LDS in whole lines; the cold part, the
// inertia and the orientation only for owners that turn or have just
// stopped turning.
// REMAP: the first step on a newly adopted set (only its overflow check
// matters here).
constexpr int FREE_WAVES = 2;    // waves per block of k_step_free
constexpr int FREE_CHUNKS = 2;   // 64-owner chunks per wave (FREE_WAVES * FREE_CHUNKS * 64 == TPB owners per block)
static_assert(FREE_WAVES * FREE_CHUNKS * 64 == TPB, "a streaming block covers the owners of one speed slot");

template <bool REMAP>
__global__ void __launch_bounds__(FREE_WAVES * 64) k_step_free(DynArgs a, RecBuf rec_out, double *q_out,
                                                              const uint8_t *oany, DevCounters *ctr)
{
    // each wave streams FREE_CHUNKS chunks of 64 consecutive owners: the
    // loads of all its chunks are issued before any chunk is computed, so a
    // wave keeps that many chunks in flight
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const int64_t No = a.n_owners;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t ob = (int64_t)lb * TPB;
    const bool rm_over = REMAP && ctr->overflow[a.rm_newbuf] != 0u;
    if (rm_over && ob + threadIdx.x == 0) ctr->stop_cd = 1u;
    const bool halt = rm_over || stopped(ctr, a.step);
    if (ob + threadIdx.x == 0) {
        if (halt) {
            halt_mark(ctr, a.step);
        } else {
            ctr->last_step_done = a.step + 1;
            ctr->contact_steps += ctr->n_contacts[a.cur];
            a.blkmax[gridDim.x] = 0.0f;   // the second kernel's blocks take their maximum here
        }
    }
    // pair skipping: the launch's first wave records the step's reach and
    // clears the speed slots the next step fills (the second kernel of the
    // step computes the same reach for itself)
    if (!halt && a.gap != 0 && lb == 0 && wv == 0) {
        const double Dn = gap_reach(a);
        if (lane == 0) a.gD[a.step & 1] = Dn;
        *gap_slot(a, a.step + 1, lane) = 0.0f;
    }
    float v2 = 0.0f, g2 = 0.0f;
    __shared__ uint4 wout[FREE_WAVES][FREE_CHUNKS][128];   // the chunks' new hot parts
    uint8_t fl[FREE_CHUNKS];
    OwnerRec rh[FREE_CHUNKS];
    // loads: flags and the hot parts of the records of every chunk, all
    // issued before any is used (consecutive lanes read consecutive 32-byte
    // hot parts: each pair of 16-byte loads covers whole lines); a stopped
    // step copies the cold parts, unchanged, straight over
#pragma unroll
    for (int c = 0; c < FREE_CHUNKS; ++c) {
        const int64_t o = ob + (int64_t)(wv * FREE_CHUNKS + c) * 64 + lane;
        fl[c] = 1u;
        rh[c] = OwnerRec{};
        if (o < No) {
            fl[c] = oany[o];
            rh[c] = load_split_hot(a.recs, o);
            if (halt) rec_out.cold[o] = a.recs.cold[o];
        }
    }
    // An owner without contacts whose record carries DEM_VOX_QSAME is
    // still: its angular velocity is zero in both record buffers (without
    // torque it stays zero) and both orientation buffers hold its
    // orientation (always true of a single sphere's identity).  Its step
    // needs neither the cold part of its record (angular velocity, mass:
    // with zero force the mass does not enter) nor its inertia nor its
    // orientation, and it writes only its hot part.  The others load their
    // cold part, inertia and template, and their orientation with them
    // (used by clumps only).  (The hot parts of owners with contacts go out
    // unchanged here and are overwritten by k_step_listed.)
#pragma unroll
    for (int c = 0; c < FREE_CHUNKS; ++c) {
        const int64_t o = ob + (int64_t)(wv * FREE_CHUNKS + c) * 64 + lane;
        const bool valid = o < No;
        OwnerRec r = rh[c];
        const bool still = !halt && !(fl[c] & 1u) && (r.vox & DEM_VOX_QSAME) != 0;
        const bool cold = valid && !halt && !(fl[c] & 1u) && !still;
        r.mass = 1.0f;   // (a still owner's: any positive value gives the same zero force term)
        OwnerAux ax{{0.0f, 0.0f, 0.0f}, -1};
        double4 qv = make_double4(1.0, 0.0, 0.0, 0.0);
        if (cold) {
            const uint4 cw = a.recs.cold[o];
            r.w[0] = __uint_as_float(cw.x);
            r.w[1] = __uint_as_float(cw.y);
            r.w[2] = __uint_as_float(cw.z);
            r.mass = __uint_as_float(cw.w);
        }
        if (valid && (halt || cold)) {
            ax = a.aux[o];
            qv = *reinterpret_cast<const double4 *>(a.q + 4 * (size_t)o);
        }
        const bool rot = valid && ax.tmpl >= 0;
        double *qo = q_out + 4 * (size_t)o;
        if (halt) {
            // a stopped step: the state is copied unchanged (the records
            // here, the orientation here; the history by k_step_listed)
            if (rot) *reinterpret_cast<double4 *>(qo) = qv;
        } else if (valid && !(fl[c] & 1u)) {
            // (a still owner: zero torque on zero angular velocity, no
            // turn; the integration of a turning path would give the same
            // bits and write back the orientation it read)
            const bool w0 = r.w[0] == 0.0f && r.w[1] == 0.0f && r.w[2] == 0.0f;
            const float inv[3] = {ax.inv_moi[0], ax.inv_moi[1], ax.inv_moi[2]};
            v2 = fmaxf(v2, advance(a, r, inv, rot, f3(0.f, 0.f, 0.f), f3(0.f, 0.f, 0.f), qv, rot ? qo : nullptr,
                                   ctr));
            if (a.gap != 0) g2 = fmaxf(g2, reach_speed2(r, a.arm));
            // after this step both record buffers hold a zero angular
            // velocity, and both orientation buffers the orientation, if
            // the owner neither turned before this step nor in it
            if (w0 && r.w[0] == 0.0f && r.w[1] == 0.0f && r.w[2] == 0.0f) r.vox |= DEM_VOX_QSAME;
            if (cold) rec_out.cold[o] = rec_cold(r);
        }
        if (valid) store_split_hot(RecBuf{wout[wv][c], nullptr}, lane, r, false);
    }
    // the hot parts go out through LDS: each store instruction then writes
    // 1 KiB of consecutive 16-byte pieces (whole lines), which non-temporal
    // stores need (a lane's own two pieces, 32 bytes apart across the wave,
    // reach memory as partial lines)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int c = 0; c < FREE_CHUNKS; ++c) {
        const int64_t ow = ob + (int64_t)(wv * FREE_CHUNKS + c) * 64;
        const uint32_t nv = ow < No ? (uint32_t)(No - ow < 64 ? No - ow : 64) : 0u;
        for (uint32_t k = lane; k < 2u * nv; k += 64u) {
            if (a.nt) st_nt(wout[wv][c][k], &rec_out.hot[2 * ow + k]);
            else rec_out.hot[2 * ow + k] = wout[wv][c][k];
        }
    }
    if (halt) return;
    __shared__ float wmax[2][FREE_WAVES];
    if (!(v2 == v2)) v2 = 3.0e38f;
    if (!(g2 == g2)) g2 = 3.0e38f;
    for (int d = 32; d > 0; d >>= 1) {
        v2 = fmaxf(v2, __shfl_xor(v2, d, 64));
        g2 = fmaxf(g2, __shfl_xor(g2, d, 64));
    }
    if (lane == 0) {
        wmax[0][wv] = v2;
        wmax[1][wv] = g2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = wmax[0][0], mg = wmax[1][0];
        for (int k = 1; k < FREE_WAVES; ++k) {
            m = fmaxf(m, wmax[0][k]);
            mg = fmaxf(mg, wmax[1][k]);
        }
        a.blkmax[lb] = m;
        // pair skipping: the block's speed bound into one of the step's
        // speed slots (non-negative floats order as their bits)
        if (a.gap != 0) atomicMax(reinterpret_cast<unsigned *>(gap_slot(a, a.step, lb)), __float_as_uint(mg));
    }
}

// The owners with contacts of a split step (see k_step_free), from the
// set's owner list (ascending: consecutive threads take consecutive owners,
// whose rows are neighbours; each entry brings the owner's first sphere and
// the bounds of its spheres' rows and B lists).  The list's length is read on the device, so
// the grid is fixed and the threads stride over the list.  The largest
// |v|^2 joins the slot after the first kernel's (an atomic maximum on the
// bits of non-negative floats, one per block).
constexpr unsigned LISTED_BLOCKS = 1024;

template <bool FACETS, bool REMAP, bool GAP>
__global__ void __launch_bounds__(TPB, 3) k_step_listed(DynArgs a, const uint4 *olist, const uint32_t *ocount,
                                                       RecBuf rec_out, double *q_out, const uint32_t *start,
                                                       const uint32_t *jarr, const uint32_t *bstart,
                                                       const uint32_t *bidx, const uint32_t *bsrc,
                                                       const uint8_t *oany, const float *hx, const float *hy,
                                                       const float *hz, const float *hw, float *ox, float *oy,
                                                       float *oz, float *ow, int64_t cap, DevCounters *ctr,
                                                       uint32_t slot)
{
    const bool rm_over = REMAP && ctr->overflow[a.rm_newbuf] != 0u;
    const bool halt = rm_over || stopped(ctr, a.step);
    const int64_t n = (int64_t)*ocount;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const HistOut ho{ox, oy, oz, ow, nullptr, 0u};
    // pair skipping: the step's reach (the first kernel of the step records
    // the same value); every lane of the wave takes part
    const double Dn = GAP && !halt ? gap_reach(a) : 0.0;
    float v2 = 0.0f, g2 = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const ListRec lr{olist[2 * i], olist[2 * i + 1]};
        const int64_t o = (int64_t)lr.h.x;
        if (halt) {
            halt_owner<false>(a, o, rec_out, q_out, start, jarr, bstart, bidx, bsrc, oany, hx, hy, hz, hw, ox, oy,
                              oz, ow, cap, ctr);
            continue;
        }
        OwnerStep st;
        owner_forces<false, FACETS, false, true, REMAP, GAP, true>(a, o, start, jarr, bstart, bidx, bsrc, oany, 0,
                                                                   hx, hy, hz, hw, ho, st, nullptr, Dn, lr);
        if (st.advance) {
            v2 = fmaxf(v2, owner_advance<false>(a, o, st, rec_out, q_out, ctr));
            if (GAP) g2 = fmaxf(g2, reach_speed2(st.r, a.arm));
        }
    }
    if (halt) return;
    __shared__ float wmax[2][TPB / 64];
    if (!(v2 == v2)) v2 = 3.0e38f;
    if (!(g2 == g2)) g2 = 3.0e38f;
    for (int d = 32; d > 0; d >>= 1) {
        v2 = fmaxf(v2, __shfl_xor(v2, d, 64));
        g2 = fmaxf(g2, __shfl_xor(g2, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wmax[0][threadIdx.x >> 6] = v2;
        wmax[1][threadIdx.x >> 6] = g2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = wmax[0][0], mg = wmax[1][0];
        for (int k = 1; k < TPB / 64; ++k) {
            m = fmaxf(m, wmax[0][k]);
            mg = fmaxf(mg, wmax[1][k]);
        }
        atomicMax(reinterpret_cast<unsigned int *>(a.blkmax + slot), __float_as_uint(m));
        if (GAP) atomicMax(reinterpret_cast<unsigned *>(gap_slot(a, a.step, blockIdx.x)), __float_as_uint(mg));
    }
}

}  // namespace

__global__ void __launch_bounds__(256) k_reduce_max(const float *blkmax, int64_t n, DevCounters *ctr)
{
    // eight independent loads in flight per thread
    float m = 0.0f;
    const int64_t bs = blockDim.x;
    int64_t i = threadIdx.x;
    for (; i + 7 * bs < n; i += 8 * bs) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = blkmax[i + k * bs];
#pragma unroll
        for (int k = 0; k < 8; ++k) m = fmaxf(m, v[k]);
    }
    for (; i < n; i += bs) m = fmaxf(m, blkmax[i]);
    for (int d = 32; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
    __shared__ float w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) ctr->maxv2[0] = __float_as_uint(fmaxf(fmaxf(w[0], w[1]), fmaxf(w[2], w[3])));
}

// Margin of the next detection under the adaptive schedule: in t = n_max h
// each geometry moves at most v t + |g| t^2 / 2 when nothing but gravity
// accelerates it (v: top speed of the last step); 10 % is added.  Capped
// by the run margin (the bins were sized for it), which is flagged.
__global__ void __launch_bounds__(64) k_adaptive_margin(DevCounters *ctr, double t, double gmag, double cap,
                                                         double vfloor)
{
    if (threadIdx.x != 0) return;
    // top sphere speed, or the fastest point of a mesh if that is faster
    const double v = fmax(sqrt((double)__uint_as_float(ctr->maxv2[0])), vfloor);
    double m = 1.1 * (v * t + 0.5 * gmag * t * t);
    uint32_t capped = 0u;
    if (!(m <= cap)) {
        m = cap;
        capped = 1u;
    }
    ctr->margin = m;
    ctr->capped = capped;
}

__global__ void __launch_bounds__(64) k_noop() {}

// Owners of fixed families: zero velocity and angular velocity, the same
// record (and orientation) in both state buffers.
__global__ void __launch_bounds__(256) k_fix_owners(RecBuf rec, RecBuf rec_alt, const double *q, double *q_alt,
                                                    const uint8_t *ofam, const uint8_t *fixed, int64_t n)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n || !fixed[ofam[o]]) return;
    OwnerRec r = load_rec(rec, o);
    for (int k = 0; k < 3; ++k) {
        r.v[k] = 0.0f;
        r.w[k] = 0.0f;
    }
    store_rec(rec, o, r);
    store_rec(rec_alt, o, r);
    *reinterpret_cast<double4 *>(q_alt + 4 * (size_t)o) = *reinterpret_cast<const double4 *>(q + 4 * (size_t)o);
}

void launch_fix_owners(RecBuf rec, RecBuf rec_alt, const double *q, double *q_alt, const uint8_t *ofam,
                       const uint8_t *fixed, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fix_owners, dim3(nblocks(n)), dim3(256), 0, s, rec, rec_alt, q, q_alt, ofam, fixed, n);
}

void launch_noop(hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    hipExtLaunchKernelGGL(k_noop, dim3(1), dim3(64), 0, s, ev0, ev1, 0);
}

void launch_adaptive_margin(DevCounters *ctr, double t, double gmag, double cap, double vfloor, hipStream_t s)
{
    hipLaunchKernelGGL(k_adaptive_margin, dim3(1), dim3(64), 0, s, ctr, t, gmag, cap, vfloor);
}

int64_t speed_slots(const DynArgs &a)
{
    return (int64_t)step_blocks(a) + 1;
}

void launch_reduce_max(const DynArgs &a, DevCounters *ctr, hipStream_t s)
{
    // (the slot after the per-block maxima holds the second kernel's of a
    // split step, and zero after any other step)
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, s, a.blkmax, (int64_t)step_blocks(a) + 1, ctr);
}

void launch_force(const DynArgs &a, AcsBuf &cur, StepBufs &sb, DevCounters *ctr, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1)
{
    auto kern = a.n_tri > 0 ? k_force<true> : k_force<false>;
    hipExtLaunchKernelGGL(kern, dim3(nblocks(a.n_spheres)), dim3(TPB), 0, s, ev0, ev1, 0, a, cur.start,
                          (const uint32_t *)cur.j, cur.hx, cur.hy, cur.hz, cur.hw, sb.aF, sb.aT, sb.bF, sb.bT,
                          sb.cap, (const DevCounters *)ctr);
}

// The step kernel for the first step on a newly adopted set (REMAP: it
// carries the history over from the previous set), for a step that also
// does a work order's first binning step (WO; single-sphere runs without
// fixed families), or for any other step.  No variant does both, nor a work
// order with clumps or fixed families: those combinations get nullptr.
using StepKernel = decltype(&k_step_fused<true, false, false, false, false, false>);
template <bool SINGLES, bool FACETS, bool FIXED, bool STAGE>
StepKernel pick_remap(bool remap, bool wo)
{
    if (wo && remap) return nullptr;
    if (wo) {
        if constexpr (SINGLES && !FIXED) return k_step_fused<SINGLES, FACETS, FIXED, STAGE, false, true>;
        return nullptr;
    }
    return remap ? k_step_fused<SINGLES, FACETS, FIXED, STAGE, true, false>
                 : k_step_fused<SINGLES, FACETS, FIXED, STAGE, false, false>;
}

bool step_is_split(const DynArgs &a, const AcsBuf &cur)
{
    return a.split && a.has_clumps && !a.has_fixed && !a.wo_keys && cur.olist;
}

bool launch_step_fused(const DynArgs &a, RecBuf rec_out, double *q_out, const AcsBuf &cur, int64_t cap,
                       DevCounters *ctr, hipStream_t s, const SplitTiming *tm)
{
    if (step_is_split(a, cur)) {
        const bool r = a.rm_start != nullptr;
        const unsigned nb = nblocks(a.n_owners);
        if (tm && tm->free0) hipEventRecord(tm->free0, s);
        hipLaunchKernelGGL(r ? k_step_free<true> : k_step_free<false>, dim3(nb), dim3(FREE_WAVES * 64), 0, s, a,
                           rec_out, q_out, (const uint8_t *)cur.oany, ctr);
        if (tm && tm->free1) hipEventRecord(tm->free1, s);
        if (tm && tm->list0) hipEventRecord(tm->list0, s);
        auto kl = a.gap != 0
                      ? (a.n_tri > 0 ? (r ? k_step_listed<true, true, true> : k_step_listed<true, false, true>)
                                     : (r ? k_step_listed<false, true, true> : k_step_listed<false, false, true>))
                      : (a.n_tri > 0 ? (r ? k_step_listed<true, true, false> : k_step_listed<true, false, false>)
                                     : (r ? k_step_listed<false, true, false> : k_step_listed<false, false, false>));
        const unsigned nl = std::min<unsigned>(nb, LISTED_BLOCKS);
        hipLaunchKernelGGL(kl, dim3(nl), dim3(TPB), 0, s, a, (const uint4 *)cur.olist,
                           (const uint32_t *)(cur.otile + owner_list_tiles(a.n_owners)), rec_out, q_out,
                           (const uint32_t *)cur.start, (const uint32_t *)cur.j, (const uint32_t *)cur.bstart,
                           (const uint32_t *)cur.bidx, (const uint32_t *)cur.bsrc, (const uint8_t *)cur.oany,
                           (const float *)cur.hx, (const float *)cur.hy, (const float *)cur.hz,
                           (const float *)cur.hw, cur.hx2, cur.hy2, cur.hz2, cur.hw2, cap, ctr, nb);
        if (tm && tm->list1) hipEventRecord(tm->list1, s);
        return true;
    }
    // runs with fixed families (mostly dormant waves) never stage
    StepKernel kern;
    const bool r = a.rm_start != nullptr, w = a.wo_keys != nullptr;
    if (a.has_fixed)
        kern = a.n_tri > 0 ? (a.has_clumps ? pick_remap<false, true, true, false>(r, w) : pick_remap<true, true, true, false>(r, w))
                           : (a.has_clumps ? pick_remap<false, false, true, false>(r, w) : pick_remap<true, false, true, false>(r, w));
    else if (a.dense_rows)
        kern = a.n_tri > 0 ? (a.has_clumps ? pick_remap<false, true, false, true>(r, w) : pick_remap<true, true, false, true>(r, w))
                           : (a.has_clumps ? pick_remap<false, false, false, true>(r, w) : pick_remap<true, false, false, true>(r, w));
    else
        kern = a.n_tri > 0 ? (a.has_clumps ? pick_remap<false, true, false, false>(r, w) : pick_remap<true, true, false, false>(r, w))
                           : (a.has_clumps ? pick_remap<false, false, false, false>(r, w) : pick_remap<true, false, false, false>(r, w));
    if (!kern) return false;
    hipLaunchKernelGGL(kern, dim3(step_blocks(a)), dim3(TPB), 0, s, a, rec_out, q_out,
                       (const uint32_t *)cur.start, (const uint32_t *)cur.j, (const uint32_t *)cur.bstart,
                       (const uint32_t *)cur.bidx, (const uint32_t *)cur.bsrc, (const uint8_t *)cur.oany,
                       (const float *)cur.hx,
                       (const float *)cur.hy, (const float *)cur.hz, (const float *)cur.hw, cur.hx2, cur.hy2,
                       cur.hz2, cur.hw2, cap, ctr);
    return true;
}

void launch_fold_integrate(const DynArgs &a, const AcsBuf &cur, StepBufs &sb, DevCounters *ctr,
                           int integrate, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    auto kern = a.has_clumps ? k_fold_integrate<false> : k_fold_integrate<true>;
    hipExtLaunchKernelGGL(kern, dim3(nblocks(a.n_owners)), dim3(TPB), 0, s, ev0, ev1, 0, a,
                          (const uint32_t *)cur.start, (const uint32_t *)cur.bstart, (const uint32_t *)cur.bidx,
                          (const float *)sb.aF, (const float *)sb.aT, (const float *)sb.bF, (const float *)sb.bT,
                          sb.cap, sb.Fo, sb.To, integrate, (const uint8_t *)cur.oany, ctr);
}
