/*
 * FP64 CPU oracle of the DEM per-timestep hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It is deliberately plain: every loop follows the
 * definition it implements, in double precision, with no blocking or fusion.
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no -ffast-math), so every
 * double operation is a separately rounded IEEE operation.
 *
 * What it computes (paper: "Chrono DEM-Engine", arXiv 2311.04648):
 *   - sphere centres of clumps from owner pose (Sec. 2.4, owner/geometry split)
 *   - the active contact set with an artificial margin (Sec. 2.1)
 *   - the history-based Hertz-Mindlin force (Sec. 4.1, Eqs. (1)-(2), and the
 *     default-model walk-through in Sec. 4.2.1)
 *   - reduction onto owners and explicit integration of the Newton-Euler
 *     equations (Sec. 4.1, Eq. (3))
 *   - contact-history carry-over when the active set is replaced (Sec. 4.2,
 *     contact wildcards are zero at birth and persist while the contact lives)
 *   - the delayed active-set schedule of Sec. 2.1 with a deterministic swap
 *     step, plus the per-step judge that counts contacts missing from the set.
 *   - sphere contacts with the facets of rigid triangle meshes under
 *     prescribed motion (Sec. 2.4: a mesh is an owner, a facet a geometry),
 *     through the closest point of each facet to the sphere centre.
 *   - family tags (Sec. 2.2.2): contacts between chosen pairs of families
 *     are never listed; owners of fixed families keep their state (the
 *     dormant elements of the active-box scheme, Sec. 6.4).
 *
 * Readings where the paper is silent (documented in the design notes):
 *   E*, G*: 1/E* = sum (1-nu^2)/E ; 1/G* = sum 2(2-nu)(1+nu)/E  (standard
 *   Hertz-Mindlin; the paper calls a helper without printing it).
 *   Contact point: middle of the overlap, c = xA - (rA - delta/2) n.
 *   Walls: plane R = inf, m = inf; cylinder side surface R = R_cyl.
 *   Integrator: semi-implicit Euler, quaternion by the exponential map,
 *   no gyroscopic term (Eq. (3) carries none).
 *   Predicates: strict '<'; pair threshold (ri + rj) + 2 m; walls r + 2 m.
 *   Parity pinned by the tests under tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n_owners, n_spheres;
    const int32_t *own_sph0;   /* [No+1] */
    const double *own_mass;    /* [No] */
    const double *own_moi;     /* [3 No] principal moments */
    const int32_t *sph_owner;  /* [Ns] */
    const double *sph_local;   /* [3 Ns] position in owner principal frame */
    const double *sph_rad;     /* [Ns] */
    const int32_t *sph_mat;    /* [Ns] */
    int64_t n_walls;
    const int32_t *wall_type;  /* 0 plane, 1 cylinder */
    const double *wall_geom;   /* [8 W] plane: p0,n ; cylinder: c,axis,R,L */
    const double *wall_vel;    /* [3 W] */
    const double *wall_omega;  /* [3 W] */
    const int32_t *wall_mat;   /* [W] */
    int64_t n_mat;
    const double *mat_E, *mat_nu;            /* [M] */
    const double *mat_cor, *mat_mu, *mat_crr; /* [M M] */
    double gravity[3];
    double h;
    int64_t n_mesh, n_tri;
    const int32_t *tri_mesh;     /* [T] mesh of each facet */
    const double *tri_local;     /* [9 T] facet vertices in the mesh frame */
    const double *mesh_origin;   /* [3 M] mesh frame origin at t = 0 (world) */
    const double *mesh_vel;      /* [3 M] constant velocity */
    const double *mesh_omega;    /* [3 M] constant angular velocity (world), about the origin */
    const int32_t *mesh_mat;     /* [M] */
    /* family tags (each may be NULL: every family 0, nothing switched off) */
    const uint8_t *owner_family; /* [No] */
    const uint8_t *wall_family;  /* [W] */
    const uint8_t *mesh_family;  /* [M] */
    const uint8_t *pair_off;     /* [256 * 256] 1: no contact between families a and b */
    const uint8_t *fixed;        /* [256] 1: owners of this family are not integrated */
} orc_sys;

static int fam_owner(const orc_sys *s, int64_t o) { return s->owner_family ? s->owner_family[o] : 0; }
static int fam_wall(const orc_sys *s, int64_t w) { return s->wall_family ? s->wall_family[w] : 0; }
static int fam_facet(const orc_sys *s, int64_t f)
{
    return s->mesh_family ? s->mesh_family[s->tri_mesh[f]] : 0;
}
/* Whether contacts between families a and b are resolved. */
static int fam_on(const orc_sys *s, int a, int b) { return !(s->pair_off && s->pair_off[256 * a + b]); }

typedef struct {
    int64_t cds;        /* contact detections run (margin > 0 or every-step) */
    int64_t swaps;      /* active sets adopted */
    int64_t misses;     /* true contacts found missing by the judge */
    int64_t repairs;    /* stale sets discarded after a miss */
    int64_t max_acs;    /* largest active set seen */
    int64_t sum_acs;    /* sum of active-set sizes over steps */
} orc_stats;

/* ------------------------------------------------------------------ */
/* rotation and sphere centres                                         */
/* ------------------------------------------------------------------ */

/* Body-to-world rotation matrix of the unit quaternion (w,x,y,z). */
static void rot_matrix(const double *q, double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void mat_vec(const double R[9], const double *v, double *out)
{
    out[0] = (R[0] * v[0] + R[1] * v[1]) + R[2] * v[2];
    out[1] = (R[3] * v[0] + R[4] * v[1]) + R[5] * v[2];
    out[2] = (R[6] * v[0] + R[7] * v[1]) + R[8] * v[2];
}

static void mat_t_vec(const double R[9], const double *v, double *out)
{
    out[0] = (R[0] * v[0] + R[3] * v[1]) + R[6] * v[2];
    out[1] = (R[1] * v[0] + R[4] * v[1]) + R[7] * v[2];
    out[2] = (R[2] * v[0] + R[5] * v[1]) + R[8] * v[2];
}

static void cross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot(const double *a, const double *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* Sphere centre = owner position + R(q) * local position (Sec. 2.4: a clump
 * owns mass and pose, its spheres carry geometry). */
void orc_sphere_centres(const orc_sys *s, const double *X, const double *q, double *xs)
{
    for (int64_t i = 0; i < s->n_spheres; ++i) {
        int64_t o = s->sph_owner[i];
        const double *p = s->sph_local + 3 * i;
        if (p[0] == 0.0 && p[1] == 0.0 && p[2] == 0.0) {
            xs[3 * i + 0] = X[3 * o + 0];
            xs[3 * i + 1] = X[3 * o + 1];
            xs[3 * i + 2] = X[3 * o + 2];
            continue;
        }
        double R[9], d[3];
        rot_matrix(q + 4 * o, R);
        mat_vec(R, p, d);
        xs[3 * i + 0] = X[3 * o + 0] + d[0];
        xs[3 * i + 1] = X[3 * o + 1] + d[1];
        xs[3 * i + 2] = X[3 * o + 2] + d[2];
    }
}

/* Pose of mesh g at step n (t = n h): origin o + v t, and the rotation by
 * the angle |w| t about the axis w / |w| (Rodrigues' rotation formula). */
static void mesh_pose(const orc_sys *s, int64_t g, int64_t step, double p[3], double R[9])
{
    double t = (double)step * s->h;
    const double *o = s->mesh_origin + 3 * g, *v = s->mesh_vel + 3 * g, *w = s->mesh_omega + 3 * g;
    for (int k = 0; k < 3; ++k) p[k] = o[k] + v[k] * t;
    double wn = sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
    if (!(wn > 0.0)) {
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    double ax = w[0] / wn, ay = w[1] / wn, az = w[2] / wn;
    double ang = wn * t;
    double c = cos(ang), sn = sin(ang), C = 1.0 - c;
    R[0] = c + ax * ax * C;
    R[1] = ax * ay * C - az * sn;
    R[2] = ax * az * C + ay * sn;
    R[3] = ay * ax * C + az * sn;
    R[4] = c + ay * ay * C;
    R[5] = ay * az * C - ax * sn;
    R[6] = az * ax * C - ay * sn;
    R[7] = az * ay * C + ax * sn;
    R[8] = c + az * az * C;
}

/* Positions of the prescribed-motion geometry at step n, in one buffer:
 * wp[3 w + k] the reference point of wall w (p0 + V n h), then from
 * wp[3 W] on the world vertices of every facet (9 per facet: origin +
 * R v for each vertex v). */
void orc_wall_positions(const orc_sys *s, int64_t step, double *wp)
{
    double t = (double)step * s->h;
    for (int64_t w = 0; w < s->n_walls; ++w)
        for (int k = 0; k < 3; ++k)
            wp[3 * w + k] = s->wall_geom[8 * w + k] + s->wall_vel[3 * w + k] * t;
    double *tw = wp + 3 * s->n_walls;
    for (int64_t g = 0; g < s->n_mesh; ++g) {
        double p[3], R[9];
        mesh_pose(s, g, step, p, R);
        for (int64_t f = 0; f < s->n_tri; ++f) {
            if (s->tri_mesh[f] != g) continue;
            for (int v = 0; v < 3; ++v) {
                const double *x = s->tri_local + 9 * f + 3 * v;
                for (int k = 0; k < 3; ++k)
                    tw[9 * f + 3 * v + k] = p[k] + ((R[3 * k] * x[0] + R[3 * k + 1] * x[1]) + R[3 * k + 2] * x[2]);
            }
        }
    }
}

static double dot3(const double *u, const double *v) { return (u[0] * v[0] + u[1] * v[1]) + u[2] * v[2]; }

/* Closest point q of the triangle (a, b, c) to p: the point of the face,
 * of an edge or a vertex, chosen by the Voronoi region of p (the standard
 * barycentric region test, e.g. Ericson, Real-Time Collision Detection,
 * 2005, Sec. 5.1.5). */
static void closest_on_tri(const double *a, const double *b, const double *c, const double *p, double *q)
{
    double ab[3], ac[3], ap[3], bp[3], cp[3];
    for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; ap[k] = p[k] - a[k]; }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) { for (int k = 0; k < 3; ++k) q[k] = a[k]; return; }
    for (int k = 0; k < 3; ++k) bp[k] = p[k] - b[k];
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) { for (int k = 0; k < 3; ++k) q[k] = b[k]; return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
        return;
    }
    for (int k = 0; k < 3; ++k) cp[k] = p[k] - c[k];
    double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
    if (d6 >= 0.0 && d5 <= d6) { for (int k = 0; k < 3; ++k) q[k] = c[k]; return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double w = d2 / (d2 - d6);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; ++k) q[k] = b[k] + w * (c[k] - b[k]);
        return;
    }
    double den = 1.0 / ((va + vb) + vc);
    double v = vb * den, w = vc * den;
    for (int k = 0; k < 3; ++k) q[k] = (a[k] + ab[k] * v) + ac[k] * w;
}

/* Exported for the tests: the closest point of triangle (a, b, c) to p,
 * and the pose of mesh g at a step. */
void orc_tri_closest(const double *a, const double *b, const double *c, const double *p, double *q)
{
    closest_on_tri(a, b, c, p, q);
}

void orc_mesh_pose(const orc_sys *s, int64_t g, int64_t step, double *p, double *R)
{
    mesh_pose(s, g, step, p, R);
}

/* Squared distance of x to facet f (world vertices tw), and the closest point. */
static double tri_dist2(const double *tw, int64_t f, const double *x, double *q)
{
    const double *v = tw + 9 * f;
    closest_on_tri(v, v + 3, v + 6, x, q);
    double dx = x[0] - q[0], dy = x[1] - q[1], dz = x[2] - q[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* ------------------------------------------------------------------ */
/* contact predicates (Sec. 2.1: every geometry is enlarged by margin m) */
/* ------------------------------------------------------------------ */

static int pair_hit(const double *xi, const double *xj, double ri, double rj, double m)
{
    double dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double T = (ri + rj) + 2.0 * m;
    return d2 < T * T;
}

static int wall_hit(const orc_sys *s, int64_t w, const double *wp, const double *x, double r, double m)
{
    const double *g = s->wall_geom + 8 * w;
    const double *p = wp + 3 * w;
    double rx = x[0] - p[0], ry = x[1] - p[1], rz = x[2] - p[2];
    if (s->wall_type[w] == 0) {
        double sd = (rx * g[3] + ry * g[4]) + rz * g[5];
        return sd < r + 2.0 * m;
    }
    double a = (rx * g[3] + ry * g[4]) + rz * g[5];
    double hl = 0.5 * g[7] + 2.0 * m;
    if (!(a <= hl && a >= -hl)) return 0;
    double px = rx - a * g[3], py = ry - a * g[4], pz = rz - a * g[5];
    double d2 = (px * px + py * py) + pz * pz;
    double T = (g[6] + r) + 2.0 * m;
    return d2 < T * T;
}

/* Sphere-facet predicate: distance below r + 2 m (strict). */
static int tri_hit(const orc_sys *s, const double *wp, int64_t f, const double *x, double r, double m)
{
    double q[3];
    double d2 = tri_dist2(wp + 3 * s->n_walls, f, x, q);
    double T = r + 2.0 * m;
    return d2 < T * T;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Brute-force active set: all sphere pairs i<j of different owners and all
 * sphere-wall pairs within the margin; keys (i<<32)|j', j' = j or Ns+w,
 * ascending.  Returns the count, or -(count) if it exceeds cap. */
int64_t orc_detect_brute(const orc_sys *s, const double *xs, const double *wp, double m,
                         uint64_t *keys, int64_t cap)
{
    int64_t n = 0;
    for (int64_t i = 0; i < s->n_spheres; ++i) {
        int fi = fam_owner(s, s->sph_owner[i]);
        for (int64_t j = i + 1; j < s->n_spheres; ++j) {
            if (s->sph_owner[i] == s->sph_owner[j]) continue;
            if (!fam_on(s, fi, fam_owner(s, s->sph_owner[j]))) continue;
            if (pair_hit(xs + 3 * i, xs + 3 * j, s->sph_rad[i], s->sph_rad[j], m)) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)j;
                ++n;
            }
        }
        for (int64_t w = 0; w < s->n_walls; ++w) {
            if (!fam_on(s, fi, fam_wall(s, w))) continue;
            if (wall_hit(s, w, wp, xs + 3 * i, s->sph_rad[i], m)) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(s->n_spheres + w);
                ++n;
            }
        }
        for (int64_t f = 0; f < s->n_tri; ++f) {
            if (!fam_on(s, fi, fam_facet(s, f))) continue;
            if (tri_hit(s, wp, f, xs + 3 * i, s->sph_rad[i], m)) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(s->n_spheres + s->n_walls + f);
                ++n;
            }
        }
    }
    return n <= cap ? n : -n;
}

typedef struct { uint64_t key; int64_t id; } binrec;

static int cmp_binrec(const void *a, const void *b)
{
    const binrec *x = a, *y = b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->id > y->id) - (x->id < y->id);
}

static uint64_t pack_bin(int64_t bx, int64_t by, int64_t bz)
{
    const int64_t off = (int64_t)1 << 20;
    return ((uint64_t)(bz + off) << 42) | ((uint64_t)(by + off) << 21) | (uint64_t)(bx + off);
}

/* Same set as orc_detect_brute, found through a uniform grid of cubic bins
 * of edge 2 (r_max + m): two spheres closer than the pair threshold always
 * lie in the same or adjacent bins.  Used for inputs too large for O(N^2). */
int64_t orc_detect_binned(const orc_sys *s, const double *xs, const double *wp, double m,
                          uint64_t *keys, int64_t cap)
{
    int64_t N = s->n_spheres;
    double rmax = 0.0;
    for (int64_t i = 0; i < N; ++i) if (s->sph_rad[i] > rmax) rmax = s->sph_rad[i];
    double b = 2.0 * (rmax + m);
    if (b <= 0.0) b = 1.0;
    binrec *br = malloc(sizeof(binrec) * (size_t)(N > 0 ? N : 1));
    int64_t *bc = malloc(sizeof(int64_t) * 3 * (size_t)(N > 0 ? N : 1));
    for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < 3; ++k) bc[3 * i + k] = (int64_t)floor(xs[3 * i + k] / b);
        br[i].key = pack_bin(bc[3 * i], bc[3 * i + 1], bc[3 * i + 2]);
        br[i].id = i;
    }
    qsort(br, (size_t)N, sizeof(binrec), cmp_binrec);
    int64_t n = 0;
    uint64_t *row = malloc(sizeof(uint64_t) * 4096);
    int64_t rowcap = 4096;
    for (int64_t i = 0; i < N; ++i) {
        int64_t nr = 0;
        int fi = fam_owner(s, s->sph_owner[i]);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    uint64_t key = pack_bin(bc[3 * i] + dx, bc[3 * i + 1] + dy, bc[3 * i + 2] + dz);
                    int64_t lo = 0, hi = N;
                    while (lo < hi) {
                        int64_t mid = (lo + hi) / 2;
                        if (br[mid].key < key) lo = mid + 1; else hi = mid;
                    }
                    for (int64_t p = lo; p < N && br[p].key == key; ++p) {
                        int64_t j = br[p].id;
                        if (j <= i || s->sph_owner[j] == s->sph_owner[i]) continue;
                        if (!fam_on(s, fi, fam_owner(s, s->sph_owner[j]))) continue;
                        if (pair_hit(xs + 3 * i, xs + 3 * j, s->sph_rad[i], s->sph_rad[j], m)) {
                            if (nr == rowcap) { rowcap *= 2; row = realloc(row, sizeof(uint64_t) * (size_t)rowcap); }
                            row[nr++] = ((uint64_t)i << 32) | (uint64_t)j;
                        }
                    }
                }
        qsort(row, (size_t)nr, sizeof(uint64_t), cmp_u64);
        for (int64_t t = 0; t < nr; ++t) {
            if (n < cap) keys[n] = row[t];
            ++n;
        }
        for (int64_t w = 0; w < s->n_walls; ++w) {
            if (!fam_on(s, fi, fam_wall(s, w))) continue;
            if (wall_hit(s, w, wp, xs + 3 * i, s->sph_rad[i], m)) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(N + w);
                ++n;
            }
        }
        for (int64_t f = 0; f < s->n_tri; ++f) {
            if (!fam_on(s, fi, fam_facet(s, f))) continue;
            if (tri_hit(s, wp, f, xs + 3 * i, s->sph_rad[i], m)) {
                if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(N + s->n_walls + f);
                ++n;
            }
        }
    }
    free(row);
    free(bc);
    free(br);
    return n <= cap ? n : -n;
}

/* The row of one sphere i: all partners j > i of other owners within the
 * margin, ascending, then the walls -- a brute-force scan over all spheres,
 * for checking sampled rows of very large inputs. Returns the row length. */
int64_t orc_detect_row(const orc_sys *s, const double *xs, const double *wp, double m, int64_t i,
                       uint64_t *keys, int64_t cap)
{
    int64_t n = 0;
    int fi = fam_owner(s, s->sph_owner[i]);
    for (int64_t j = i + 1; j < s->n_spheres; ++j) {
        if (s->sph_owner[i] == s->sph_owner[j]) continue;
        if (!fam_on(s, fi, fam_owner(s, s->sph_owner[j]))) continue;
        if (pair_hit(xs + 3 * i, xs + 3 * j, s->sph_rad[i], s->sph_rad[j], m)) {
            if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)j;
            ++n;
        }
    }
    for (int64_t w = 0; w < s->n_walls; ++w) {
        if (!fam_on(s, fi, fam_wall(s, w))) continue;
        if (wall_hit(s, w, wp, xs + 3 * i, s->sph_rad[i], m)) {
            if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(s->n_spheres + w);
            ++n;
        }
    }
    for (int64_t f = 0; f < s->n_tri; ++f) {
        if (!fam_on(s, fi, fam_facet(s, f))) continue;
        if (tri_hit(s, wp, f, xs + 3 * i, s->sph_rad[i], m)) {
            if (n < cap) keys[n] = ((uint64_t)i << 32) | (uint64_t)(s->n_spheres + s->n_walls + f);
            ++n;
        }
    }
    return n;
}

/* Number of true contacts (margin 0) absent from the sorted set `acs`. */
int64_t orc_count_missing(const orc_sys *s, const double *xs, const double *wp,
                          const uint64_t *acs, int64_t n_acs, uint64_t *scratch, int64_t cap)
{
    int64_t nt = orc_detect_binned(s, xs, wp, 0.0, scratch, cap);
    if (nt < 0) return -1;
    int64_t miss = 0, p = 0;
    for (int64_t t = 0; t < nt; ++t) {
        while (p < n_acs && acs[p] < scratch[t]) ++p;
        if (!(p < n_acs && acs[p] == scratch[t])) ++miss;
    }
    return miss;
}

/* ------------------------------------------------------------------ */
/* contact history carry-over (Sec. 4.2: wildcards are zero at birth)  */
/* History per contact: tangential displacement (3) and contact age.    */
/* ------------------------------------------------------------------ */

void orc_remap(const uint64_t *old_keys, const double *old_hist, int64_t n_old,
               const uint64_t *new_keys, double *new_hist, int64_t n_new)
{
    int64_t p = 0;
    for (int64_t c = 0; c < n_new; ++c) {
        while (p < n_old && old_keys[p] < new_keys[c]) ++p;
        if (p < n_old && old_keys[p] == new_keys[c]) {
            for (int k = 0; k < 4; ++k) new_hist[4 * c + k] = old_hist[4 * p + k];
        } else {
            for (int k = 0; k < 4; ++k) new_hist[4 * c + k] = 0.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Hertz-Mindlin contact force (Sec. 4.1 Eqs. (1)-(2); Sec. 4.2.1)      */
/* ------------------------------------------------------------------ */

static void pair_moduli(const orc_sys *s, int ma, int mb, double *Estar, double *Gstar)
{
    double Ea = s->mat_E[ma], na = s->mat_nu[ma], Eb = s->mat_E[mb], nb = s->mat_nu[mb];
    *Estar = 1.0 / ((1.0 - na * na) / Ea + (1.0 - nb * nb) / Eb);
    *Gstar = 1.0 / (2.0 * (2.0 - na) * (1.0 + na) / Ea + 2.0 * (2.0 - nb) * (1.0 + nb) / Eb);
}

/* Velocity of the material point of owner o currently at world arm r
 * (= point - owner centre): V + R (w_body x R^T r). */
static void point_velocity(const double *V, const double *Wb, const double *q, const double *arm,
                           double *out)
{
    double R[9], loc[3], rv[3], rw[3];
    rot_matrix(q, R);
    mat_t_vec(R, arm, loc);
    cross(Wb, loc, rv);
    mat_vec(R, rv, rw);
    out[0] = V[0] + rw[0];
    out[1] = V[1] + rw[1];
    out[2] = V[2] + rw[2];
}

/* Evaluates every contact of the set on the state (X,q,V,W) at `step`.
 *   hist  [4n] in/out tangential micro-displacement and contact age
 *         (the contact wildcards of the default model)
 *   Fc    [3n] force on geometry A (world); B receives -Fc
 *   TcA   [3n] torque on owner A about its centre; TcB [3n] on owner B
 *   Fo,To [3No] per-owner sums; Fw [3W] force on each wall (may be NULL)
 *   touch [n]  1 if the pair is in contact (may be NULL)                 */
/* How long a contact's first impact lasts, the phase in which rolling
 * resistance does not act (the default model's walk-through, Sec. 4.2.1):
 * the contact as a mass m on the linear spring k = (4/3) E* Re^(1/2) and
 * dashpot c = -2 sqrt((5/3) m E*) beta Re^(1/4), Re = sqrt(R_bar) (the
 * walk-through's simplified constants), rebounds after half a period of its
 * damped oscillation, pi / w_d, w_d^2 = k/m - (c/(2m))^2.  An overdamped
 * contact has no rebound: -1 (the resistance acts at once). */
static double first_impact_duration(double Estar, double beta, double Rbar, double m)
{
    double Re = sqrt(Rbar);
    double k = 4.0 / 3.0 * Estar * sqrt(Re);
    double c = -2.0 * sqrt(5.0 / 3.0 * m * Estar) * beta * pow(Re, 0.25);
    double half = c / (2.0 * m);
    double wd2 = k / m - half * half;
    return wd2 > 0.0 ? M_PI / sqrt(wd2) : -1.0;
}

/* Mindlin's tangential spring-dashpot for a contact (Sec. 4.1 Eq. (2)):
 * stiffness k_t = 8 G* sqrt(R_bar delta), damping c_t = 2 sqrt(5/6) |beta|
 * sqrt(m k_t), force f = -k_t xi - c_t u_t.  Where |f| exceeds the Coulomb
 * limit the force is scaled to the limit and the stored displacement is
 * moved to where the spring-dashpot gives that force (reading R3); a force
 * below 1e-12 N is dropped.  Writes f, updates xi, returns |k_t xi| + |c_t| vsum
 * (vsum: the magnitudes the relative velocity is summed from). */
static double mindlin_tangential(double Gstar, double beta, double sqrtRd, double m, double limit,
                                 const double *ut, double vsum, double *xi, double *f)
{
    double kt = 8.0 * Gstar * sqrtRd;
    double ct = -2.0 * sqrt(5.0 / 6.0) * beta * sqrt(m * kt);
    double spring[3], damper[3];
    for (int k = 0; k < 3; ++k) {
        spring[k] = -kt * xi[k];
        damper[k] = -ct * ut[k];
        f[k] = spring[k] + damper[k];
    }
    double terms = sqrt(dot(spring, spring)) + fabs(ct) * vsum;
    double fmag = sqrt(dot(f, f));
    if (!(fmag > 1e-12)) {
        f[0] = f[1] = f[2] = 0.0;
        return terms;
    }
    if (fmag > limit) {
        for (int k = 0; k < 3; ++k) {
            f[k] *= limit / fmag;
            xi[k] = -(f[k] + ct * ut[k]) / kt;
        }
    }
    return terms;
}

void orc_forces(const orc_sys *s, const double *X, const double *q, const double *V,
                const double *Wb, int64_t step, const uint64_t *keys, int64_t n, double *hist,
                double *Fc, double *TcA, double *TcB, double *Fo, double *To, double *Fw,
                int32_t *touch, double *scale)
{
    int64_t Ns = s->n_spheres, No = s->n_owners;
    double *xs = malloc(sizeof(double) * 3 * (size_t)(Ns > 0 ? Ns : 1));
    double *wp = malloc(sizeof(double) * (size_t)(3 * s->n_walls + 9 * s->n_tri + 1));
    orc_sphere_centres(s, X, q, xs);
    orc_wall_positions(s, step, wp);
    memset(Fo, 0, sizeof(double) * 3 * (size_t)No);
    memset(To, 0, sizeof(double) * 3 * (size_t)No);
    if (Fw) memset(Fw, 0, sizeof(double) * 3 * (size_t)s->n_walls);
    const double h = s->h;
    for (int64_t c = 0; c < n; ++c) {
        int64_t i = (int64_t)(keys[c] >> 32), jp = (int64_t)(keys[c] & 0xffffffffu);
        int64_t oA = s->sph_owner[i];
        const double *xA = xs + 3 * i;
        double rA = s->sph_rad[i];
        double *xi = hist + 4 * c;
        double nrm[3], delta, Rbar, mbar, XB[3];
        int matB, is_wall = jp >= Ns, oB = -1;
        int touching = 0;
        if (!is_wall) {
            const double *xB = xs + 3 * jp;
            double rB = s->sph_rad[jp];
            double dx = xA[0] - xB[0], dy = xA[1] - xB[1], dz = xA[2] - xB[2];
            double d2 = (dx * dx + dy * dy) + dz * dz;
            double T = rA + rB;
            touching = d2 < T * T;
            if (touching) {
                double d = sqrt(d2);
                nrm[0] = dx / d; nrm[1] = dy / d; nrm[2] = dz / d;
                delta = T - d;
                Rbar = rA * rB / (rA + rB);
                oB = s->sph_owner[jp];
                mbar = s->own_mass[oA] * s->own_mass[oB] / (s->own_mass[oA] + s->own_mass[oB]);
                matB = s->sph_mat[jp];
            }
        } else if (jp >= Ns + s->n_walls) {
            /* facet of a mesh: normal from the closest point to the centre,
             * the facet seen as flat (R = rA), the mesh as of infinite mass */
            int64_t f = jp - Ns - s->n_walls;
            double qf[3];
            double d2 = tri_dist2(wp + 3 * s->n_walls, f, xA, qf);
            touching = d2 < rA * rA && d2 > 0.0;
            if (touching) {
                double d = sqrt(d2);
                nrm[0] = (xA[0] - qf[0]) / d; nrm[1] = (xA[1] - qf[1]) / d; nrm[2] = (xA[2] - qf[2]) / d;
                delta = rA - d;
                Rbar = rA;
                mbar = s->own_mass[oA];
                int64_t g = s->tri_mesh[f];
                matB = s->mesh_mat[g];
                double R9[9];
                mesh_pose(s, g, step, XB, R9);
            }
        } else {
            int64_t w = jp - Ns;
            const double *g = s->wall_geom + 8 * w;
            const double *p = wp + 3 * w;
            double rx = xA[0] - p[0], ry = xA[1] - p[1], rz = xA[2] - p[2];
            if (s->wall_type[w] == 0) {
                double sd = (rx * g[3] + ry * g[4]) + rz * g[5];
                touching = sd < rA;
                if (touching) {
                    nrm[0] = g[3]; nrm[1] = g[4]; nrm[2] = g[5];
                    delta = rA - sd;
                    Rbar = rA;
                }
            } else {
                double a = (rx * g[3] + ry * g[4]) + rz * g[5];
                double hl = 0.5 * g[7];
                double px = rx - a * g[3], py = ry - a * g[4], pz = rz - a * g[5];
                double d2 = (px * px + py * py) + pz * pz;
                double T = g[6] + rA;
                touching = (a <= hl && a >= -hl) && d2 < T * T && d2 > 0.0;
                if (touching) {
                    double d = sqrt(d2);
                    nrm[0] = px / d; nrm[1] = py / d; nrm[2] = pz / d;
                    delta = T - d;
                    Rbar = rA * g[6] / (rA + g[6]);
                }
            }
            if (touching) {
                mbar = s->own_mass[oA];
                matB = s->wall_mat[w];
                for (int k = 0; k < 3; ++k) XB[k] = p[k];
            }
        }
        if (touch) touch[c] = touching;
        if (scale) scale[c] = 0.0;
        if (!touching) {
            /* false positive of the margin: zero force, history released */
            for (int k = 0; k < 3; ++k) {
                xi[k] = 0.0; Fc[3 * c + k] = 0.0; TcA[3 * c + k] = 0.0; TcB[3 * c + k] = 0.0;
            }
            xi[3] = 0.0;
            continue;
        }
        int matA = s->sph_mat[i];
        double Estar, Gstar;
        pair_moduli(s, matA, matB, &Estar, &Gstar);
        double cor = s->mat_cor[matA * s->n_mat + matB];
        double mu = s->mat_mu[matA * s->n_mat + matB];
        double crr = s->mat_crr[matA * s->n_mat + matB];

        /* contact point: middle of the overlap region */
        double cp[3], armA[3], armB[3], vA[3], vB[3];
        for (int k = 0; k < 3; ++k) cp[k] = xA[k] - (rA - 0.5 * delta) * nrm[k];
        for (int k = 0; k < 3; ++k) armA[k] = cp[k] - X[3 * oA + k];
        point_velocity(V + 3 * oA, Wb + 3 * oA, q + 4 * oA, armA, vA);
        if (!is_wall) {
            for (int k = 0; k < 3; ++k) { XB[k] = X[3 * oB + k]; armB[k] = cp[k] - XB[k]; }
            point_velocity(V + 3 * oB, Wb + 3 * oB, q + 4 * oB, armB, vB);
        } else {
            /* wall or mesh: prescribed velocity plus rotation about its
             * reference point */
            const int facet = jp >= Ns + s->n_walls;
            const double *wv = facet ? s->mesh_vel + 3 * s->tri_mesh[jp - Ns - s->n_walls] : s->wall_vel + 3 * (jp - Ns);
            const double *ww = facet ? s->mesh_omega + 3 * s->tri_mesh[jp - Ns - s->n_walls]
                                     : s->wall_omega + 3 * (jp - Ns);
            double rotv[3];
            for (int k = 0; k < 3; ++k) armB[k] = cp[k] - XB[k];
            cross(ww, armB, rotv);
            for (int k = 0; k < 3; ++k) vB[k] = wv[k] + rotv[k];
        }
        /* relative velocity of A w.r.t. B, split along the normal */
        double VBl[3];
        if (!is_wall) {
            for (int k = 0; k < 3; ++k) VBl[k] = V[3 * oB + k];
        } else if (jp >= Ns + s->n_walls) {
            for (int k = 0; k < 3; ++k) VBl[k] = s->mesh_vel[3 * s->tri_mesh[jp - Ns - s->n_walls] + k];
        } else {
            for (int k = 0; k < 3; ++k) VBl[k] = s->wall_vel[3 * (jp - Ns) + k];
        }
        double u[3], ut[3];
        for (int k = 0; k < 3; ++k) u[k] = vA[k] - vB[k];
        double pn = dot(u, nrm);
        for (int k = 0; k < 3; ++k) ut[k] = u[k] - pn * nrm[k];
        /* history: add h v_t, then project onto the tangent plane (Eq. (2));
         * the contact ages by one step */
        for (int k = 0; k < 3; ++k) xi[k] = xi[k] + h * ut[k];
        double xin = dot(xi, nrm);
        for (int k = 0; k < 3; ++k) xi[k] = xi[k] - xin * nrm[k];
        xi[3] = xi[3] + h;
        /* normal spring-damper */
        double sqrtRd = sqrt(Rbar * delta);
        double Sn = 2.0 * Estar * sqrtRd;
        double loge = (cor < 1e-12) ? log(1e-12) : log(cor);
        double beta = loge / sqrt(loge * loge + M_PI * M_PI);
        double kn = 2.0 / 3.0 * Sn;
        double gn = 2.0 * sqrt(5.0 / 6.0) * beta * sqrt(Sn * mbar);
        double F[3];
        for (int k = 0; k < 3; ++k) F[k] = (kn * delta + gn * pn) * nrm[k];
        /* magnitudes of what the force sums (for the rounding bound of a
         * float evaluation): the normal spring, and the dampers acting on a
         * relative velocity summed from parts of these magnitudes */
        double vsum = 0.0;
        {
            double rA[3], rB[3];
            for (int k = 0; k < 3; ++k) { rA[k] = vA[k] - V[3 * oA + k]; rB[k] = vB[k] - VBl[k]; }
            vsum = sqrt(dot(V + 3 * oA, V + 3 * oA)) + sqrt(dot(rA, rA)) + sqrt(dot(VBl, VBl)) + sqrt(dot(rB, rB));
        }
        double mag = fabs(kn * delta) + fabs(gn) * vsum;
        /* rolling resistance (Sec. 4.1 Eq. (2), Sec. 4.3.1): a torque-only
         * force of magnitude C_rr |F| along the rolling part of the relative
         * velocity at the contact point, once the contact has outlasted its
         * first impact (reading R4) */
        double Fr[3] = {0.0, 0.0, 0.0};
        if (crr > 0.0 && xi[3] > first_impact_duration(Estar, beta, Rbar, mbar)) {
            double wrA[3], wrB[3], vr[3];   /* rotational parts of vA and vB */
            for (int k = 0; k < 3; ++k) { wrA[k] = vA[k] - V[3 * oA + k]; wrB[k] = vB[k] - VBl[k]; }
            for (int k = 0; k < 3; ++k) vr[k] = wrB[k] - wrA[k];
            double vrn = sqrt(dot(vr, vr));
            if (vrn > 1e-12) {
                double fmag = sqrt(dot(F, F));
                for (int k = 0; k < 3; ++k) Fr[k] = (crr * fmag) * (vr[k] / vrn);
            }
        }
        /* Mindlin tangential force (Sec. 4.1 Eq. (2)) under the Coulomb
         * limit (reading R3) */
        if (mu > 0.0) {
            double ft[3];
            mag += mindlin_tangential(Gstar, beta, sqrtRd, mbar, mu * sqrt(dot(F, F)), ut, vsum, xi, ft);
            for (int k = 0; k < 3; ++k) F[k] += ft[k];
        }
        if (scale) scale[c] = mag;
        double tA[3], tB[3], mF[3] = {-F[0], -F[1], -F[2]};
        double FA_t[3] = {F[0] + Fr[0], F[1] + Fr[1], F[2] + Fr[2]};
        double FB_t[3] = {-FA_t[0], -FA_t[1], -FA_t[2]};
        cross(armA, FA_t, tA);
        cross(armB, FB_t, tB);
        for (int k = 0; k < 3; ++k) {
            Fc[3 * c + k] = F[k]; TcA[3 * c + k] = tA[k]; TcB[3 * c + k] = tB[k];
            Fo[3 * oA + k] += F[k];
            To[3 * oA + k] += tA[k];
        }
        if (!is_wall) {
            for (int k = 0; k < 3; ++k) { Fo[3 * oB + k] += mF[k]; To[3 * oB + k] += tB[k]; }
        } else if (Fw && jp < Ns + s->n_walls) {
            for (int k = 0; k < 3; ++k) Fw[3 * (jp - Ns) + k] += mF[k];
        }
    }
    free(wp);
    free(xs);
}

/* ------------------------------------------------------------------ */
/* explicit integration (Sec. 4.1, Eq. (3))                            */
/* ------------------------------------------------------------------ */

static void quat_mul(const double *a, const double *b, double *o)
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Semi-implicit Euler: velocities first, then positions with the new
 * velocities; orientation by the exponential map of h * w_body.  Owners of
 * fixed families keep their state. */
void orc_integrate(const orc_sys *s, double *X, double *q, double *V, double *Wb,
                   const double *Fo, const double *To)
{
    const double h = s->h;
    for (int64_t o = 0; o < s->n_owners; ++o) {
        if (s->fixed && s->fixed[fam_owner(s, o)]) continue;
        double m = s->own_mass[o];
        for (int k = 0; k < 3; ++k) V[3 * o + k] += h * (Fo[3 * o + k] / m + s->gravity[k]);
        double R[9], tb[3];
        rot_matrix(q + 4 * o, R);
        mat_t_vec(R, To + 3 * o, tb);
        for (int k = 0; k < 3; ++k) Wb[3 * o + k] += h * (tb[k] / s->own_moi[3 * o + k]);
        for (int k = 0; k < 3; ++k) X[3 * o + k] += h * V[3 * o + k];
        double th[3] = {h * Wb[3 * o], h * Wb[3 * o + 1], h * Wb[3 * o + 2]};
        double ang = sqrt(dot(th, th));
        if (ang > 0.0) {
            double dq[4], nq[4];
            double sh = sin(0.5 * ang) / ang;
            dq[0] = cos(0.5 * ang); dq[1] = sh * th[0]; dq[2] = sh * th[1]; dq[3] = sh * th[2];
            quat_mul(q + 4 * o, dq, nq);
            double nn = sqrt(nq[0] * nq[0] + nq[1] * nq[1] + nq[2] * nq[2] + nq[3] * nq[3]);
            for (int k = 0; k < 4; ++k) q[4 * o + k] = nq[k] / nn;
        }
    }
}

/* ------------------------------------------------------------------ */
/* delayed active-set schedule (Sec. 2.1) with the per-step judge       */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t *keys; double *hist; int64_t n; } acs_buf;

static int64_t detect_into(const orc_sys *s, const double *X, const double *q, int64_t step,
                           double m, uint64_t *keys, int64_t cap, double *xs, double *wp)
{
    orc_sphere_centres(s, X, q, xs);
    orc_wall_positions(s, step, wp);
    return orc_detect_binned(s, xs, wp, m, keys, cap);
}

/* Runs n_steps steps.  mode 0: detection every step with margin 0.
 * mode 1: a work order (state snapshot) every k steps, its active set
 * (margin m) adopted lam steps later (0 <= lam <= k); the very first set is
 * detected synchronously.  judge: count true contacts missing from the set
 * in use before each force evaluation; a miss discards that set and detects
 * again synchronously from the current state (nothing has been integrated
 * with the incomplete set yet).
 * acs_keys/acs_hist/acs_n carry the set and its history in and out.
 * Returns 0, or -1 if cap is too small.                                  */
int orc_run(const orc_sys *s, double *X, double *q, double *V, double *Wb, int64_t *step,
            int64_t n_steps, int mode, int64_t k, int64_t lam, double m, int judge,
            uint64_t *acs_keys, double *acs_hist, int64_t *acs_n, int64_t cap, orc_stats *st)
{
    int64_t Ns = s->n_spheres, No = s->n_owners, W = s->n_walls;
    double *xs = malloc(sizeof(double) * 3 * (size_t)(Ns > 0 ? Ns : 1));
    double *wp = malloc(sizeof(double) * (size_t)(3 * W + 9 * s->n_tri + 1));
    double *Fo = malloc(sizeof(double) * 3 * (size_t)(No > 0 ? No : 1));
    double *To = malloc(sizeof(double) * 3 * (size_t)(No > 0 ? No : 1));
    double *Fc = malloc(sizeof(double) * 3 * (size_t)cap);
    double *TA = malloc(sizeof(double) * 3 * (size_t)cap);
    double *TB = malloc(sizeof(double) * 3 * (size_t)cap);
    uint64_t *tmp = malloc(sizeof(uint64_t) * (size_t)cap);
    acs_buf cur = {malloc(sizeof(uint64_t) * (size_t)cap), malloc(sizeof(double) * 4 * (size_t)cap), *acs_n};
    acs_buf pend = {malloc(sizeof(uint64_t) * (size_t)cap), malloc(sizeof(double) * 4 * (size_t)cap), 0};
    acs_buf fresh = {malloc(sizeof(uint64_t) * (size_t)cap), malloc(sizeof(double) * 4 * (size_t)cap), 0};
    memcpy(cur.keys, acs_keys, sizeof(uint64_t) * (size_t)cur.n);
    memcpy(cur.hist, acs_hist, sizeof(double) * 4 * (size_t)cur.n);
    int rc = 0, pending = 0;
    int64_t pend_swap = 0, next_wo = *step;
    double mm = (mode == 0) ? 0.0 : m;
    if (mode == 0) { k = 1; lam = 0; }
    for (int64_t t = 0; t < n_steps; ++t) {
        int64_t n = *step;
        int adopt = 0;
        if (t == 0 && mode == 1) {
            /* the first set of a run is detected synchronously */
            fresh.n = detect_into(s, X, q, n, mm, fresh.keys, cap, xs, wp);
            if (fresh.n < 0) { rc = -1; break; }
            st->cds++;
            adopt = 1;
            next_wo = n + k;
        } else {
            if (pending && n == pend_swap) {
                memcpy(fresh.keys, pend.keys, sizeof(uint64_t) * (size_t)pend.n);
                fresh.n = pend.n;
                pending = 0;
                adopt = 1;
            }
            if (n == next_wo) {
                pend.n = detect_into(s, X, q, n, mm, pend.keys, cap, xs, wp);
                if (pend.n < 0) { rc = -1; break; }
                st->cds++;
                pending = 1;
                pend_swap = n + lam;
                next_wo = n + k;
                if (lam == 0) {
                    memcpy(fresh.keys, pend.keys, sizeof(uint64_t) * (size_t)pend.n);
                    fresh.n = pend.n;
                    pending = 0;
                    adopt = 1;
                }
            }
        }
        if (judge && mode == 1) {
            const uint64_t *cand = adopt ? fresh.keys : cur.keys;
            int64_t cn = adopt ? fresh.n : cur.n;
            orc_sphere_centres(s, X, q, xs);
            orc_wall_positions(s, n, wp);
            int64_t miss = orc_count_missing(s, xs, wp, cand, cn, tmp, cap);
            if (miss < 0) { rc = -1; break; }
            if (miss > 0) {
                st->misses += miss;
                st->repairs++;
                fresh.n = orc_detect_binned(s, xs, wp, mm, fresh.keys, cap);
                if (fresh.n < 0) { rc = -1; break; }
                st->cds++;
                adopt = 1;
                pending = 0;
                next_wo = n + k;
            }
        }
        if (adopt) {
            orc_remap(cur.keys, cur.hist, cur.n, fresh.keys, fresh.hist, fresh.n);
            acs_buf tswap = cur; cur = fresh; fresh = tswap;
            st->swaps++;
        }
        if (cur.n > st->max_acs) st->max_acs = cur.n;
        st->sum_acs += cur.n;
        orc_forces(s, X, q, V, Wb, n, cur.keys, cur.n, cur.hist, Fc, TA, TB, Fo, To, NULL, NULL, NULL);
        orc_integrate(s, X, q, V, Wb, Fo, To);
        *step = n + 1;
    }
    if (rc == 0) {
        memcpy(acs_keys, cur.keys, sizeof(uint64_t) * (size_t)cur.n);
        memcpy(acs_hist, cur.hist, sizeof(double) * 4 * (size_t)cur.n);
        *acs_n = cur.n;
    }
    free(cur.keys); free(cur.hist); free(pend.keys); free(pend.hist);
    free(fresh.keys); free(fresh.hist);
    free(tmp); free(TB); free(TA); free(Fc); free(To); free(Fo); free(wp); free(xs);
    return rc;
}
