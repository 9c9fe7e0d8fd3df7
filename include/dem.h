/*
 * dem.h -- C ABI of the MI355X (gfx950) DEM hot-path library.
 *
 * The operations follow the paper "Chrono DEM-Engine: A Discrete Element
 * Method dual-GPU simulator with customizable contact forces and element
 * shape" (arXiv 2311.04648):
 *   - problem statement (materials, clump templates, analytic walls, time
 *     step, gravity, divergence velocity): Sec. 3 (sample script);
 *   - owner / geometry hierarchy (clumps own mass, spheres carry geometry and
 *     material): Sec. 2.4;
 *   - delayed active-contact-set update with an artificial margin and the
 *     bound n_max on the steps run without a new set: Sec. 2.1;
 *   - history-based Hertz-Mindlin contact force: Sec. 4.1, Eqs. (1)-(2) and
 *     the default-model walk-through of Sec. 4.2.1;
 *   - reduction of sphere contact forces onto owners and explicit
 *     integration of the Newton-Euler equations: Sec. 4.1, Eq. (3);
 *   - compressed positions (integer voxel index + sub-voxel offset): Sec. 2.3
 *     (this library keeps the integer voxel index and stores the sub-voxel
 *     offset as a 32-bit float on a fixed 2^-38 m grid).
 *
 * Conventions for every entry point:
 *   - Return value: a dem_status; DEM_OK (0) on success.  Nothing throws
 *     across the ABI.  dem_last_error(ctx) returns a message for the last
 *     failure on that context (valid until the next call on it).
 *   - Memory: the caller owns all device memory.  dem_workspace_size reports
 *     how many bytes of device memory one binding needs; the caller allocates
 *     one buffer of at least that size (256-byte aligned) and hands it to
 *     dem_bind.  The library never frees caller memory.  The library itself
 *     allocates only its opaque host context, a few bytes of pinned host
 *     memory for read-backs, HIP events, and, with meshes, pinned staging
 *     for the per-step mesh poses (64 KiB per mesh), and nothing else.
 *   - Host arrays (const double*, float* ...) are plain host pointers; they
 *     are read or written before the call returns.
 *   - Streams: dem_stream is a hipStream_t passed as void* (NULL = the
 *     default stream).  Calls that take a stream enqueue their device work on
 *     it; results in device memory are valid after that stream is
 *     synchronised.  Calls that return values to host memory synchronise the
 *     stream they use before returning.
 *   - Sizes are element counts unless stated as bytes.  Arrays with a
 *     leading factor (e.g. [3*No]) are row-major: element k of item i is at
 *     3*i + k.
 */
#ifndef DEM_H
#define DEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *dem_stream;
typedef struct dem_ctx dem_ctx;

typedef enum {
    DEM_OK = 0,
    DEM_ERR_ARG = 1,       /* invalid argument (message in dem_last_error) */
    DEM_ERR_CAPACITY = 2,  /* contact array too small; required size reported */
    DEM_ERR_HIP = 3,       /* a HIP runtime call failed */
    DEM_ERR_DIVERGED = 4,  /* NaN or speed above v_error_out (Sec. 3, SetErrorOutVelocity) */
    DEM_ERR_MISSED = 5,    /* judge found a missing contact and repair is disabled */
    DEM_ERR_STATE = 6      /* call out of order (e.g. step before bind) */
} dem_status;

typedef enum {
    DEM_CD_EVERY = 0,      /* contact detection every step, margin 0 */
    DEM_CD_FIXED = 1,      /* delayed detection every cd_interval steps, Sec. 2.1 */
    DEM_CD_LEARNED = 2,    /* delayed detection, interval chosen by the MLP */
    DEM_CD_ADAPTIVE = 3    /* Sec. 2.1's own policy: a work order goes out at every
                              adoption, so detection is always in flight; its latency
                              lambda (steps) is adapted from the measured timing of past
                              cycles to the smallest value at which the dynamics stream
                              does not wait; the margin follows from n_max = 2 lambda
                              steps, the current top speed and gravity
                              (m = 1.1 (v t + |g| t^2 / 2), t = n_max dt), capped by
                              params.margin (when the cap binds, lambda shrinks) */
} dem_cd_mode;

enum { DEM_WALL_PLANE = 0, DEM_WALL_CYLINDER = 1 };

/* Material table (Sec. 3, LoadMaterial; Sec. 4.2.1): Young's modulus and
 * Poisson ratio per material; restitution, friction and rolling-resistance
 * coefficients per material pair ([n*n], row a, column b). */
typedef struct {
    int32_t n;
    const double *E, *nu;
    const double *cor, *mu, *crr;
} dem_materials;

/* Clump templates (Sec. 3, LoadClumpType; Sec. 2.4): template t has the
 * component spheres sph_begin[t] .. sph_begin[t+1]-1, whose positions
 * sph_pos[3*k..] are given in the template's principal frame relative to
 * its mass centre.  Positions must be float32-representable. */
typedef struct {
    int32_t n;
    const int32_t *sph_begin;   /* [n+1] */
    const double *sph_pos;      /* [3*sph_begin[n]] */
} dem_templates;

/* Analytic walls with prescribed motion (Sec. 3, InstructBoxDomainBoundingBC,
 * AddCylinder; Sec. 2.2.2 prescribed motion).  geom[8*w..]:
 *   plane:    p0.xyz, unit normal (pointing into the granular domain), -, -
 *   cylinder: centre.xyz, unit axis, radius, length (side surface only)
 * The reference point moves as p(n) = p0 + vel * (n * dt); omega only sets
 * the surface velocity of a cylinder. */
typedef struct {
    int32_t n;
    const int32_t *type;        /* [n] DEM_WALL_* */
    const double *geom;         /* [8*n] */
    const double *vel;          /* [3*n] */
    const double *omega;        /* [3*n] */
    const int32_t *mat;         /* [n] */
} dem_walls;

/* Rigid triangle meshes with prescribed motion (Sec. 2.4: a mesh is an owner
 * whose geometries are triangle facets; Sec. 5 drives a bladed mixer at a
 * constant angular velocity).  Facet f belongs to mesh tri_mesh[f]; its three
 * vertices tri_local[9*f .. 9*f+8] (x,y,z each) are given in the mesh frame.
 * At step n (t = n dt) mesh g is the rotation by the angle |omega_g| t about
 * the axis omega_g / |omega_g| (Rodrigues' formula, evaluated on the host in
 * FP64), followed by the translation origin_g + vel_g t; its surface moves
 * with vel_g + omega_g x (x - p_g(t)).  A facet acts on a sphere like a flat
 * wall of infinite mass (Sec. 4.2.1 with R = r and m = m_sphere) along the
 * line from the closest point of the facet to the sphere centre. */
#define DEM_MAX_MESHES 4
typedef struct {
    int32_t n_mesh;             /* 0 .. DEM_MAX_MESHES */
    int64_t n_tri;              /* facets */
    const int32_t *tri_mesh;    /* [n_tri] */
    const double *tri_local;    /* [9*n_tri] */
    const double *origin;       /* [3*n_mesh] reference point at step 0 */
    const double *vel;          /* [3*n_mesh] */
    const double *omega;        /* [3*n_mesh] rad/s, world frame, about the reference point */
    const int32_t *mat;         /* [n_mesh] */
} dem_meshes;

/* Owners (clumps or single spheres) and their spheres (Sec. 2.4).  Spheres are
 * numbered owner-major: owner o has spheres own_sph0[o] .. own_sph0[o+1]-1.
 * own_tmpl[o] = -1 marks a single sphere at the owner's centre (isotropic
 * inertia); otherwise sph_comp[s] is the index of sphere s among that
 * template's components.  Masses, inertias and radii must be
 * float32-representable. */
typedef struct {
    int64_t n_owners, n_spheres;
    const int32_t *own_sph0;    /* [No+1] */
    const int32_t *own_tmpl;    /* [No] */
    const double *own_mass;     /* [No] */
    const double *own_moi;      /* [3*No] principal moments */
    const int32_t *sph_comp;    /* [Ns] */
    const double *sph_rad;      /* [Ns] */
    const int32_t *sph_mat;     /* [Ns] */
} dem_bodies;

/* Run parameters (Sec. 3: SetInitTimeStep, SetGravitationalAcceleration,
 * SetErrorOutVelocity; Sec. 2.1: margin and update interval). */
typedef struct {
    double gravity[3];
    double dt;
    double margin;          /* per-geometry margin m; a pair is listed if its gap < 2m */
    double v_error_out;     /* divergence speed (0 = off) */
    double domain_lo[3];    /* box that holds every sphere centre */
    double domain_hi[3];
    int32_t cd_mode;        /* dem_cd_mode */
    int32_t cd_interval;    /* k: steps between work orders (FIXED) */
    int32_t cd_latency;     /* lambda: steps from work order to adoption, 0 <= lambda <= k
                               (ADAPTIVE: the first lambda, >= 1) */
    int32_t judge;          /* 1: count contacts missing from the set in use, every step */
    int32_t repair;         /* 1: a missed contact discards the stale set (default) */
    int32_t cd_interval_max;/* LEARNED: upper bound on the interval; ADAPTIVE: on lambda */
    int32_t timing;         /* n > 0: time kernel stages with HIP events (stats->stage_ms);
                               the dynamics kernels are sampled every n-th step */
    double mlp_safety;      /* LEARNED: factor on the predicted horizon (0 = 1) */
    int32_t bin_sort;       /* sort of (bin, sphere id): 0 one pass over the bin histogram
                               (default), 1 stable LSD radix sort with 8-bit digits;
                               both give the same order */
    int32_t dyn_path;       /* dem_step's dynamics: 0 one fused kernel per step (default:
                               each owner evaluates its A-row contacts and re-evaluates
                               its B-side contacts with the same function, then
                               integrates; state and history are double-buffered),
                               1 two kernels (forces with per-contact reactions, then
                               the ordered fold and integration); 2 and 3 the fused
                               kernel with its history writes always (2) or never (3)
                               gathered per wave in LDS, which 0 decides from the last
                               contact count read back (at least one per two spheres:
                               gathered); 4 in clump systems without fixed families, a
                               streaming kernel over every owner plus a kernel over the
                               owners with contacts (0 picks it for sparse sets); all
                               give the same bits */
    int32_t no_pair_skip;   /* 0 (default): in single-sphere systems without fixed
                               families, a dense set's pairs proven apart are skipped by
                               the fused step (each pair keeps a lower bound of its gap,
                               the step a bound of how far any two surfaces can have
                               closed in since; such a pair cannot touch, and the step
                               gives it exactly what evaluating it would: no force, zero
                               history); nonzero: every pair is evaluated every step.
                               Both give the same bits. */
} dem_params;

/* Statistics of a dem_step call (Sec. 2.1, thread collaboration stats). */
typedef struct {
    int64_t steps;          /* steps completed */
    int64_t step;           /* global step counter after the call */
    int64_t cds;            /* contact detections launched */
    int64_t swaps;          /* active sets adopted */
    int64_t misses;         /* true contacts found missing (judge on) */
    int64_t repairs;        /* sets discarded after a miss */
    int64_t n_contacts;     /* size of the active set in use at the end */
    int64_t required_capacity; /* on DEM_ERR_CAPACITY: contacts needed */
    double max_speed;       /* largest owner speed seen at the last step */
    double ms;              /* wall time of the call */
    double mean_interval;   /* mean steps between work orders */
    /* with params.timing: summed device time and launch count per stage,
     * measured with HIP events on the stream the stage runs on:
     * [0] force kernel and [1] fold + integrate kernel of the two-kernel
     * dynamics (one event pair per kernel, every `timing`-th step), or [1]
     * the fused step kernel (runs of 4 back-to-back launches between one
     * event pair, one run per `timing` steps, placed where the next 4 steps
     * have no other dynamics-stream work); [2] contact detection (bin, sort,
     * detect, B lists); [3] history remap; [4] an empty one-wave kernel
     * bracketed like [0]/[1] (one per event pair of [0]/[1]: the markers'
     * own overhead, so stage_ms[1] - stage_ms[4] is kernel time) */
    double stage_ms[5];
    int64_t stage_n[5];
    double mean_contacts;   /* mean size of the active set over the steps */
} dem_step_stats;

/* Creates a context for one problem: the set-up of the sample script of
 * Sec. 3 (materials, clump templates, box walls and analytic objects, time
 * step, gravity, divergence speed) over the owner / geometry hierarchy of
 * Sec. 2.4, with the margin and update interval of Sec. 2.1.  Copies every
 * array it is given (host pointers, read before the call returns); the
 * context is owned by the caller and released with dem_destroy.  Derives
 * the detection bins (cubes of edge 2 (r_max + margin), enlarged by a
 * relative 1e-6) and the voxel origin.
 * Errors: DEM_ERR_ARG on inconsistent sizes or values (message in
 * dem_last_error(NULL) when no context is returned). */
dem_status dem_create(const dem_params *params, const dem_materials *mats,
                      const dem_templates *tmpls, const dem_walls *walls,
                      const dem_bodies *bodies, dem_ctx **out);

/* Installs the meshes of a context (Sec. 2.4, Sec. 5); call between
 * dem_create and dem_bind (the workspace holds per-facet buffers).  Copies
 * the arrays; replaces earlier meshes; NULL or n_mesh = 0 removes them.
 * Contact partners of a sphere then include facets, with keys
 * j' = n_spheres + n_walls + f.
 * Errors: DEM_ERR_STATE after dem_bind; DEM_ERR_ARG on counts out of range,
 * a facet of an unknown mesh, a material out of range or a non-finite
 * value. */
dem_status dem_set_meshes(dem_ctx *ctx, const dem_meshes *meshes);

/* Family tags (Sec. 2.2.2) and the active-box scheme built on them
 * (Sec. 6.4).  Every owner, wall and mesh carries a family 0..255.
 * Contacts between the families of a switched-off pair are never listed
 * (detection, judge).  Owners of fixed families are never integrated and
 * keep zero velocity (this call and dem_set_state set their v and w to 0);
 * they still touch the owners of other families, as static bodies.  The
 * active box of the paper: the owners outside the box go to a fixed family
 * whose pair with itself is switched off.  Arrays (each may be NULL: all 0):
 * owner_family [n_owners], wall_family [n_walls], mesh_family [n_mesh],
 * pair_off [256*256] (1 switches the pair (a, b) off; must be symmetric),
 * fixed [256] (1 fixes a family). */
typedef struct {
    const uint8_t *owner_family;
    const uint8_t *wall_family;
    const uint8_t *mesh_family;
    const uint8_t *pair_off;
    const uint8_t *fixed;
} dem_families;

/* Installs family tags (after dem_bind; call again to move an active box).
 * If a state is set, the fixed owners' velocities are zeroed and the
 * current set is rebuilt at once with the run margin (the history of pairs
 * still listed is carried over; a pending delayed detection is dropped).
 * Synchronises the stream.
 * Errors: DEM_ERR_STATE before dem_bind; DEM_ERR_ARG on an asymmetric or
 * non-0/1 pair table; DEM_ERR_CAPACITY if the rebuilt set does not fit. */
dem_status dem_set_families(dem_ctx *ctx, const dem_families *fam, dem_stream stream);

/* Device bytes one binding needs for a contact array of contact_capacity
 * entries (per active-set buffer).  The paper keeps the whole state, both
 * active contact sets (the one in use and the one the kinematics side
 * builds, Sec. 2.1) and their contact history (Sec. 4.2) resident on the
 * GPUs; this is the size of that residency here: owner state x2, sphere
 * records, two active sets with history x2, detection workspaces for the
 * two streams, counters.  Writes *bytes; no device work.
 * Errors: DEM_ERR_ARG (negative capacity, null pointer). */
dem_status dem_workspace_size(const dem_ctx *ctx, int64_t contact_capacity, int64_t *bytes);

/* Binds caller-owned device memory (>= dem_workspace_size bytes, 256-byte
 * aligned; the library carves it and never frees it) and uploads the
 * constant tables of the problem (Sec. 3: materials as the pairwise
 * contact parameters of Sec. 4.2.1, templates of Sec. 2.4, walls).
 * Re-binding drops the state and the contact set; set them again
 * afterwards.  Synchronous (the uploads finish before it returns).
 * Errors: DEM_ERR_ARG (null or misaligned pointer, too few bytes),
 * DEM_ERR_HIP. */
dem_status dem_bind(dem_ctx *ctx, void *device_workspace, int64_t bytes, int64_t contact_capacity);

/* Uploads a state (the owner kinematics of Sec. 2.4, Sec. 4.1; positions in
 * the compressed form of Sec. 2.3): X [3*No] world positions (m), q [4*No] unit quaternions
 * (w,x,y,z; body to world), v [3*No] velocities, w [3*No] angular velocities
 * in the body frame.  Positions are stored as voxel index + float offset on
 * a 2^-38 m grid; X that lie on that grid are stored exactly.  Single-sphere
 * owners keep their angular velocity in the world frame (their orientation
 * has no physical effect), so their q is ignored and read back as
 * identity.  Clears the step counter to `step` and the contact set. */
dem_status dem_set_state(dem_ctx *ctx, const double *X, const double *q, const float *v,
                         const float *w, int64_t step, dem_stream stream);

/* Reads the state back (Sec. 2.4 owner kinematics; positions decoded from
 * the Sec. 2.3 voxel form exactly to FP64; same layout as dem_set_state; w
 * of clumps in the body frame, of single spheres in the world frame with
 * q = identity).  Host output arrays (any may be NULL); synchronises the
 * stream.  Errors: DEM_ERR_STATE before a state is set, DEM_ERR_HIP. */
dem_status dem_get_state(dem_ctx *ctx, double *X, double *q, float *v, float *w,
                         int64_t *step, dem_stream stream);

/* Sphere binning, the first stage of contact detection (Sec. 2.1 and the
 * binning method the paper cites in Sec. 1): a uniform grid of cubic bins of
 * edge 2 (r_max + margin); sphere centres (Sec. 2.4: owner position plus
 * the rotated template offset), bin keys and a stable sort of
 * (key, sphere id); errors DEM_ERR_STATE before a state is set.
 * Optional read-back to host arrays (NULL to skip): keys [Ns] and ids [Ns] in
 * sorted order; synchronises the stream when reading back. */
dem_status dem_bin(dem_ctx *ctx, dem_stream stream, uint32_t *sorted_keys, uint32_t *sorted_ids);

/* Contact detection on the current state with margin m (0 <= m <= params
 * margin) (Sec. 2.1): every sphere pair of different owners with
 * |xi - xj|^2 < ((ri + rj) + 2m)^2, every sphere-wall pair with gap < 2m
 * and every sphere-facet pair with |xi - closest point|^2 < (ri + 2m)^2, as
 * sorted keys (i << 32) | j' (j' = j, n_spheres + wall index, or
 * n_spheres + n_walls + facet index).  The
 * new set replaces the current one; contact history of pairs present in both
 * is carried over, new pairs start from zero (Sec. 4.2).  If n_contacts is
 * not NULL the stream is synchronised and the set size written there.
 * Errors: DEM_ERR_CAPACITY (n_contacts receives the size needed). */
dem_status dem_detect_contacts(dem_ctx *ctx, double margin, dem_stream stream,
                               int64_t *n_contacts);

/* Evaluates the Hertz-Mindlin force of every contact in the current set and
 * reduces forces and torques onto owners (Sec. 4.1), without integrating.
 * Updates the contact history as a step would.  Results via dem_get_forces. */
dem_status dem_forces(dem_ctx *ctx, dem_stream stream);

/* Reads the last dem_forces results: the owner sums of Sec. 4.1 Eq. (3)
 * F_owner, T_owner [3*No] (world frame, torque about the owner centre) and
 * the per-contact force of Eqs. (1)-(2) F_contact [3*n] (force on geometry
 * A of each contact, in set order; cap = its capacity in contacts).  Host
 * arrays, any may be NULL.  Synchronises the stream.
 * Errors: DEM_ERR_STATE before dem_forces, DEM_ERR_CAPACITY if cap is
 * below the set size. */
dem_status dem_get_forces(dem_ctx *ctx, float *F_owner, float *T_owner, float *F_contact,
                          int64_t cap, dem_stream stream);

/* Advances n_steps steps of force, reduction and integration with the
 * contact-detection schedule of params.cd_mode (Sec. 2.1).  `dyn` carries
 * the dynamics work; `kin` the delayed detection (may equal dyn).  Stats
 * may be NULL.  Synchronises both streams before returning.
 * Errors: DEM_ERR_CAPACITY, DEM_ERR_DIVERGED (state frozen at the failing
 * step, reported in stats->step), DEM_ERR_MISSED (judge on, repair off). */
dem_status dem_step(dem_ctx *ctx, int64_t n_steps, dem_stream dyn, dem_stream kin,
                    dem_step_stats *stats);

/* Reads the current active contact set (Sec. 2.1) with its contact history
 * (the tangential displacement and contact age that the default model keeps
 * per contact, Sec. 4.2.1): keys [cap] and history [4*cap] (float:
 * tangential displacement xyz, contact age in seconds; the age is tracked
 * only when some material pair has rolling resistance, else reads 0).
 * n receives the set size; DEM_ERR_CAPACITY if cap is smaller. */
dem_status dem_get_contacts(dem_ctx *ctx, uint64_t *keys, float *hist, int64_t cap,
                            int64_t *n, dem_stream stream);

/* Installs an active contact set (Sec. 2.1; strictly ascending keys as
 * dem_detect_contacts produces) with its history (Sec. 4.2.1) ([4*n] as dem_get_contacts; NULL = zero).  Errors: DEM_ERR_ARG on bad keys,
 * DEM_ERR_CAPACITY if n exceeds the bound capacity. */
dem_status dem_set_contacts(dem_ctx *ctx, const uint64_t *keys, const float *hist, int64_t n,
                            dem_stream stream);

/* Counts true contacts (margin 0) absent from the current set -- the judge
 * of the delayed schedule: Sec. 2.1 requires that the margin cover every
 * contact that can form before the next set arrives, so a set in use
 * must hold every pair that touches; this counts the pairs for which it
 * does not.  Synchronises; writes the count to *missing.
 * Errors: DEM_ERR_STATE before a state and a set exist, DEM_ERR_HIP. */
dem_status dem_count_missing(dem_ctx *ctx, dem_stream stream, int64_t *missing);

/* ---- learned contact-detection interval ---------------------------------
 * A 6-32-32-1 tanh MLP predicts, per feature cell, log(1 + the number of
 * steps) a contact set detected now stays complete (labels censored at
 * DEM_MLP_KCAP).  Parameters are 1313 floats in the
 * order W1[32x6], b1[32], W2[32x32], b2[32], W3[1x32], b3[1] (row-major,
 * out x in). */
#define DEM_MLP_NPARAM 1313
#define DEM_MLP_NFEAT 6
#define DEM_MLP_KCAP 1024   /* label horizon K (steps) used by the features */

/* Installs MLP parameters used by DEM_CD_LEARNED: the learned replacement
 * of the update bound n_max of Sec. 2.1.  params is a host array of
 * DEM_MLP_NPARAM floats, copied into the context (and to device memory once
 * bound); NULL removes the model, and the learned schedule then uses its
 * analytic fallback.  Errors: DEM_ERR_ARG on a non-finite value,
 * DEM_ERR_HIP. */
dem_status dem_mlp_set(dem_ctx *ctx, const float *params);

/* Computes the per-cell features of the current state relative to the
 * snapshot of the set in use (device pointer out [ncell_cap*6] floats,
 * row-major) and returns the number of occupied cells in *ncell. */
dem_status dem_features(dem_ctx *ctx, float *out_dev, int64_t ncell_cap, int64_t *ncell,
                        dem_stream stream);

/* Stand-alone MLP kernels on caller device buffers (row-major float32):
 *   forward:  X [n*6] -> Y [n]
 *   backward: dL/dparams for the expectile loss of Y against targets T [n]
 *             with asymmetry tau, written to grad [1313] (mean over n), and
 *             the loss to loss[0]; summed in a fixed order (deterministic).
 *   adam:     one Adam step on params (device) with moments m, v [1313]. */
dem_status dem_mlp_forward(const float *params_dev, const float *X_dev, float *Y_dev, int64_t n,
                           dem_stream stream);
dem_status dem_mlp_backward(const float *params_dev, const float *X_dev, const float *T_dev,
                            int64_t n, float tau, float *grad_dev, float *loss_dev,
                            float *work_dev, int64_t work_bytes, dem_stream stream);
dem_status dem_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                        int64_t t, float lr, float beta1, float beta2, float eps,
                        dem_stream stream);
/* Device bytes of the `work` buffer dem_mlp_backward needs for n samples. */
int64_t dem_mlp_backward_work_bytes(int64_t n);

/* dem_mlp_backward without the work buffer, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training or
 * serving loops, harnesses that forbid allocation).  The per-block partial
 * gradients live in a fixed array inside the library, one copy per GPU,
 * held from the first use until the process ends: 4,036,608 bytes on each device,
 * enough for n <= DEM_MLP_NOALLOC_MAX samples.  No hipMalloc or other
 * allocating call is made; the array's device address is looked up once per
 * device (with that device current) at the first call.  Same kernels and
 * summation order as dem_mlp_backward, so the results are the same bits.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams or host threads) race; calls on one stream are
 * ordered and safe.  Errors: DEM_ERR_ARG (n <= 0, a null pointer, tau
 * outside (0, 1)), DEM_ERR_CAPACITY (n > DEM_MLP_NOALLOC_MAX), DEM_ERR_HIP;
 * the message is in dem_last_error(NULL). */
#define DEM_MLP_NOALLOC_MAX 49152
dem_status dem_mlp_backward_noalloc(const float *params_dev, const float *X_dev, const float *T_dev,
                                    int64_t n, float tau, float *grad_dev, float *loss_dev,
                                    dem_stream stream);

/* ---- training-log tools (the learned interval is trained on logs the
 * method generates with per-step detection) ------------------------------
 * dem_snapshot: copies the current state into the reference that features
 *   are measured against (steps since the last detection restart there; in
 *   DEM_CD_LEARNED runs every work order does this).
 * dem_feature_cells: after dem_features, the feature-cell id of each output
 *   row (host cell_ids [cap]) and of each owner (host owner_cell [No]).
 * dem_label_begin: detects, with the run margin, a side "label" set on the
 *   current state (not used by the dynamics); n_contacts receives its size.
 * dem_label_update: on the current state, every true contact (margin 0)
 *   absent from the label set lowers first_miss_dev[cell] (device uint32
 *   per feature cell, cells of both owners) to t with an atomic minimum.
 * dem_info: grid sizes: vals[0..7] = bins, feature cells, nx, ny, nz,
 *   radix bits, contact capacity, step. */
dem_status dem_snapshot(dem_ctx *ctx, dem_stream stream);
dem_status dem_feature_cells(dem_ctx *ctx, uint32_t *cell_ids, int64_t cap, uint32_t *owner_cell,
                             int64_t *n_cells_total, dem_stream stream);
dem_status dem_label_begin(dem_ctx *ctx, dem_stream stream, int64_t *n_contacts);
dem_status dem_label_update(dem_ctx *ctx, uint32_t t, uint32_t *first_miss_dev, dem_stream stream);
dem_status dem_info(const dem_ctx *ctx, int64_t *vals, int64_t n);

/* Message of the last failure on ctx; with ctx = NULL, of the last failed
 * context-free call (the MLP kernels) on the calling host thread. */
const char *dem_last_error(const dem_ctx *ctx);
void dem_destroy(dem_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
