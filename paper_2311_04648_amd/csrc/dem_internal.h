// Internal declarations shared by the HIP kernels and the host side of the
// DEM library (gfx950).  Device data layout:
//   owners   records (RecBuf): in clump systems two arrays, hot parts
//            (voxel word, offsets, velocity: 32 B per owner) and cold parts
//            (angular velocity, mass: 16 B), so a stream over owners at rest
//            moves hot parts only; in single-sphere systems whole 48 B
//            records, so a gather of a contact partner reads one record;
//            OwnerAux[No] (inverse inertia + template), double4 q[No]
//   spheres  SphRec[Ns] (owner, radius, material, template component)
//   contacts per active-set buffer: acs_start[Ns+1] (CSR by lower sphere
//            id), acs_j[cap] (partner: sphere id, Ns + wall index, or Ns + W + facet),
//            hist x/y/z [cap] (SoA float), B-side lists bstart/bidx
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEM_VOXEL_SIZE (1.0 / 16384.0)          // 2^-14 m
#define DEM_VOXEL_INV 16384.0
#define DEM_OFF_QUANT_INV 274877906944.0        // 2^38
#define DEM_OFF_QUANT (1.0 / 274877906944.0)    // 2^-38 m
#define DEM_OFF_STEPS 16777216.0                // 2^24 offset steps per voxel
#define DEM_VOX_BITS 21
#define DEM_VOX_MASK ((1ull << 21) - 1ull)
#define DEM_NO_COMP 0xffffffffu

struct __align__(16) OwnerRec {
    uint64_t vox;      // voxel index, 3 x 21 bits (x low)
    float off[3];      // offset inside the voxel, multiples of 2^-38 m
    float v[3];        // velocity (m/s)
    float w[3];        // angular velocity: body frame (clumps) / world frame (single spheres)
    float mass;
};
static_assert(sizeof(OwnerRec) == 48, "owner record must be 48 bytes");

// Owner records in device memory (OwnerRec is their form in registers).
// Clump systems: two arrays, the hot parts (voxel word, offsets, velocity:
// the record's first 32 bytes, hot[2 o] and hot[2 o + 1]) and the cold
// parts (angular velocity, mass: cold[o]).  Single-sphere systems, whose
// steps gather whole partner records: one array of whole records,
// hot[3 o .. 3 o + 2], cold null.  A wave's 64 records staged in LDS take
// the layout of the array they come from (rec_lds).
struct RecBuf {
    uint4 *hot;
    uint4 *cold;
};

// Whether the streams over a system's state (each step's records, a
// detection's candidate records, the learned interval's snapshot) are
// stored non-temporally: when the state is larger than the last-level
// cache (256 MB), a stream is not read back from a cache anyway, and
// normal stores would evict data that is.
inline bool stream_nt(int64_t n_owners) { return n_owners * 48 > (int64_t)256 << 20; }

struct __align__(16) OwnerAux {
    float inv_moi[3];
    int32_t tmpl;      // -1: single sphere at the owner centre
};

// Reference state of the learned-interval features: an owner's position
// and velocity at the previous feature pass (the features measure motion
// since then).
struct __align__(16) SnapRec {
    uint64_t vox;
    float off[3];
    float v[3];
};
static_assert(sizeof(SnapRec) == 32, "snapshot record must be 32 bytes");

struct __align__(16) SphRec {
    uint32_t owner;
    float rad;
    uint32_t mat;
    uint32_t tcomp;    // index into the template component table, DEM_NO_COMP for single spheres
};

struct __align__(16) MatPair {
    float Estar, Gstar, beta, mu;
    float crr;         // rolling-resistance coefficient
    float kns, tcol;   // simplified stiffness and collision time of the rolling-resistance gate (unused: per contact)
    float pad;
};

struct __align__(16) WallDev {
    double geom[8];
    double vel[3];
    double omega[3];
    int32_t type;
    int32_t mat;
    int32_t family;
};

// A facet of a rigid mesh: vertices in the mesh frame, mesh index.
struct __align__(16) TriDev {
    double v[9];
    int32_t mesh;
    int32_t pad;
};

// Pose of a mesh at one step (computed on the host) and its rigid motion.
struct MeshPose {
    double p[3];       // reference point
    double R[9];       // rotation, row-major
    float vel[3];      // velocity of the reference point
    float omega[3];    // angular velocity (world)
    int32_t mat;
    int32_t family;
};

constexpr int MAX_MESHES = 4;

struct MeshPoses {
    MeshPose m[MAX_MESHES];
};

// A facet at the pose of one detection: world vertices, their box, and the
// range of bins whose spheres may touch it (bins cx0 .. cx0 + ncx - 1, etc.).
struct __align__(16) FacetDev {
    double v[9];
    double lo[3], hi[3];
    int32_t cx0, ncx, cy0, ncy, cz0, ncz;
    int32_t family, pad[3];
};

// Candidate record in bin-sorted order: exact FP64 centre, radius, sphere id.
struct __align__(16) Cand {
    double x, y, z;
    float r;
    uint32_t id;
};

struct Grid {
    double lo[3];
    double inv_b;
    int32_t nx, ny, nz;
    uint32_t nbins;
};

struct Origin {
    double o[3];
};

// Device counters (one block of device memory).
struct DevCounters {
    uint32_t n_contacts[2];   // size of each active-set buffer
    uint32_t overflow[2];     // detection into buffer b overflowed
    uint32_t required;        // largest set size asked for
    uint32_t stop_cd;         // set at a swap when the adopted set overflowed
    uint32_t div[2];          // divergence seen by the integrator, by step parity
    uint32_t miss;            // judge: missing true contacts
    uint32_t maxv2[4];        // max |v|^2 bits per step slot
    uint32_t capped;          // adaptive schedule: the derived margin hit its cap
    int64_t last_step_done;
    uint32_t ncell;           // feature cells in use
    uint32_t pad1;
    unsigned long long contact_steps;   // sum over integrated steps of the set size in use
    double margin;            // adaptive schedule: margin of the next detection
};

struct ScanTmp {
    uint32_t *partials;  // >= 2 scan_tmp_elems(n) entries
};

// ---------------------------------------------------------------------------
// host-side launchers (implemented in the .hip files)
// ---------------------------------------------------------------------------
int64_t scan_tmp_elems(int64_t n);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s);
void launch_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n, hipStream_t s);
// exclusive scan of in[0..n) into out[0..n], out[n] = total (in may equal
// out); optionally also into out2, and with ctr set, the total is recorded as
// the size of active-set buffer `buf` and checked against cap.
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *partials,
                        hipStream_t s, uint32_t *out2 = nullptr, DevCounters *ctr = nullptr,
                        int64_t cap = 0, int buf = 0);
// two scans of the same length in one pair of launches (partials holds
// 2 scan_tmp_elems(n) entries); the first may check its total against cap
void scan_exclusive_u32_pair(const uint32_t *in0, uint32_t *out0, uint32_t *out0b, DevCounters *ctr, int64_t cap,
                             int buf, const uint32_t *in1, uint32_t *out1, uint32_t *out1b, int64_t n,
                             uint32_t *partials, hipStream_t s);
void launch_zero3(uint32_t *p0, int64_t n0, uint32_t *p1, int64_t n1, uint32_t *p2, int64_t n2, hipStream_t s);
int64_t radix_hist_elems(int64_t n);
// stable LSD radix sort of (keys, vals) on the low `bits` bits; the buffer
// pairs are swapped as needed so the result ends in (*keys, *vals); the alt
// buffers are scratch of the same size.
void radix_sort_u32(uint32_t **keys, uint32_t **vals, uint32_t **keys_alt, uint32_t **vals_alt,
                    int64_t n, int bits, uint32_t *hist, uint32_t *partials, hipStream_t s);

struct DetectArgs {
    RecBuf recs;
    const double *q;        // 4 per owner
    const OwnerAux *aux;
    const SphRec *sph;
    const float *tpos;      // 4 per template component
    const WallDev *walls;
    int32_t n_walls;
    int64_t n_spheres;
    Grid grid;
    Origin org;
    double margin;
    const double *margin_dev;   // if set, the margin is read from device memory
    const uint32_t *own_sph0;   // [No+1] first sphere of each owner (null: one sphere per owner)
    const uint2 *sph_range;     // [Ns] per sphere its owner's sphere range (null with own_sph0)
    int64_t n_owners;
    double h;
    int64_t step;
    double rmax;            // largest sphere radius
    const TriDev *tri;      // [n_tri] facets of the meshes
    int32_t n_tri;
    MeshPoses poses;        // mesh poses at `step`
    const uint8_t *ofam;    // [No] family of each owner
    const uint8_t *pairoff; // [256*256] 1: contacts between the two families are not listed (null: none)
    const uint8_t *famfixed;// [256] 1: owners of the family are fixed
    // dormant families (fixed, and switched off with every fixed family and
    // every wall and mesh family): their spheres are left out of the binning
    // of each detection; the active spheres find them in a static index
    // built when the tags or the state are set (null: none)
    const uint8_t *famdormant;      // [256]
    const uint32_t *dcell_start;    // [nbins+1] bin ranges of the dormant index
    const Cand *dcand;              // dormant candidates in bin order
    const float4 *dcandf;           // their FP32 copies for the prefilter
    int32_t owner_list;     // build the owner list of each set written (AcsBuf::olist)
    int32_t nt;             // store the binning's streams non-temporally (stream_nt)
};

struct CdWork {
    uint32_t *keys, *vals, *keys_alt, *vals_alt;   // sorted result lands in keys/vals
    uint32_t *rank;        // [Ns] each binned sphere's slot among its bin's spheres (from the counting)
    Cand *cand_tmp, *cand;
    float4 *candf;         // [Ns] bin order: FP32 centre relative to the grid origin, radius
    uint32_t *cell_count, *cell_start;
    uint32_t *count;       // [Ns+1]
    uint32_t *stage;       // [16 Ns] staged partners of the single-traversal detection
    uint32_t *hist, *partials;
    FacetDev *fac;         // [n_tri] facets at the pose of the detection
    uint32_t *frow;        // [n_tri + 1] bin rows per facet, then their offsets
    int sort_bits;
    int sort_mode;         // 0: one-pass bin sort, 1: 8-bit LSD radix passes
};

// A listed owner's record (AcsBuf::olist): {owner, first sphere s0, the row
// start and the B-list start of s0}, then the row and B-list lengths of its
// spheres as bytes (.x: rows of spheres 0-3; .y: rows of 4-5 in the low
// half, B lists of 0-1 in the high half; .z: B lists of 2-5) and in .w the
// sphere count, or LIST_NOPACK for an owner of more than LIST_SPHERES
// spheres or with a row or B list longer than 255.
constexpr uint32_t LIST_SPHERES = 6;
constexpr uint32_t LIST_NOPACK = 0xffffffffu;

struct AcsBuf {
    uint32_t *start;   // [Ns+1]
    uint32_t *j;       // [cap]
    float *hx, *hy, *hz;
    float *hw;         // contact age (tracked only with rolling resistance)
    // second history buffer: the fused step reads (hx..hw) and writes these,
    // then the two are swapped
    float *hx2, *hy2, *hz2, *hw2;
    uint32_t *bstart;  // [Ns+1]
    uint32_t *bidx;    // [cap] contact index of each B-list entry
    uint32_t *bsrc;    // [cap] the A sphere of that contact
    uint32_t *bcur;    // [Ns+1] scratch cursor
    uint8_t *oany;     // [No] bit 0: any sphere of the owner has a row or B-list entry in this set;
                       // bit 1: the owner is in a fixed family
    // the owners with bit 0 set, ascending (built with the flags in clump
    // systems without fixed families, where a step with a sparse set runs
    // them in a kernel of their own), as two uint4 each (see LIST_SPHERES);
    // their count is otile[owner_list_tiles(No)]
    uint4 *olist;      // [2 No]
    uint32_t *otile;   // [owner_list_tiles(No) + 1] per-tile offsets, then the count
    // single-sphere systems: per contact a lower bound of the pair's gap
    // plus the reach of the chain it was written in (DynArgs::gap); null
    // in clump systems
    float *gk;         // [cap]
};

// tiles of the owner-list compaction
int64_t owner_list_tiles(int64_t n_owners);

inline void swap_hist(AcsBuf &b)
{
    float *t;
    t = b.hx; b.hx = b.hx2; b.hx2 = t;
    t = b.hy; b.hy = b.hy2; b.hy2 = t;
    t = b.hz; b.hz = b.hz2; b.hz2 = t;
    t = b.hw; b.hw = b.hw2; b.hw2 = t;
}

void launch_bin(const DetectArgs &a, CdWork &w, hipStream_t s, uint32_t *z1 = nullptr, int64_t n1 = 0,
                uint32_t *z2 = nullptr, int64_t n2 = 0, bool order_bins = true);
// full detection into `out` (count, scan, write, sort rows, B lists)
void launch_detect(const DetectArgs &a, CdWork &w, AcsBuf &out, int64_t cap, DevCounters *ctr,
                   int buf, hipStream_t s);
// the same in two parts: the front reads the owner state (centres, bin
// keys, candidate records, bin counts; w.cell_count must hold zeros, as the
// back leaves it); the back reads only what the front wrote, so it may run
// on another stream after an event
void launch_detect_front(const DetectArgs &a, CdWork &w, AcsBuf &out, hipStream_t s);
void launch_detect_back(const DetectArgs &a, CdWork &w, AcsBuf &out, int64_t cap, DevCounters *ctr,
                        int buf, hipStream_t s);
void launch_judge(const DetectArgs &a, CdWork &w, const AcsBuf &cur, int64_t cap, DevCounters *ctr,
                  hipStream_t s);
// the static index of the dormant spheres (a.famdormant must be set):
// cell ranges into dcell_start, candidates into dcand / dcandf; w supplies
// scratch (keys, cell_count, partials)
void launch_dormant_index(const DetectArgs &a, CdWork &w, uint32_t *dcell_start, Cand *dcand, float4 *dcandf,
                          hipStream_t s);
void launch_blists(AcsBuf &b, int64_t n_spheres, int64_t cap, uint32_t *partials, hipStream_t s);
// the per-owner contact flags of a set (AcsBuf::oany) from its rows and B
// lists (an overflowed set flags nothing)
// With `list`, also the list of the owners with contacts (AcsBuf::olist;
// `partials` is scan scratch).
void launch_owner_flags(AcsBuf &b, const uint32_t *own_sph0, int64_t n_owners, int64_t n_spheres, int64_t cap,
                        const uint8_t *ofam, const uint8_t *fixed, hipStream_t s, bool list = false,
                        uint32_t *partials = nullptr);
void launch_owner_list(AcsBuf &b, const uint32_t *own_sph0, int64_t n_owners, uint32_t *partials, hipStream_t s);
void launch_remap(const AcsBuf &oldb, AcsBuf &newb, int64_t n_spheres, DevCounters *ctr, int newbuf,
                  int rolling, hipStream_t s);

struct DynArgs {
    RecBuf recs;
    double *q;
    const OwnerAux *aux;
    const float *inv_i;     // per owner: isotropic inverse moment of inertia (single spheres)
    const uint32_t *own_sph0;
    const SphRec *sph;
    const float *tpos;
    const WallDev *walls;
    const MatPair *mat;
    int32_t n_mat;
    int32_t n_walls;
    int64_t n_owners, n_spheres;
    Origin org;
    double h;
    float g[3];
    float v_err2;
    int64_t step;
    int32_t has_clumps;
    int32_t rolling;        // some material pair has rolling resistance
    int32_t cur;            // active-set buffer in use (for statistics)
    float *blkmax;          // per-block max |v|^2 of the last integration [ceil(No/256)]
    const TriDev *tri;      // [n_tri] facets of the meshes
    int32_t n_tri;
    const MeshPose *poses;  // [MAX_MESHES] mesh poses at `step` (device memory; null without meshes)
    int32_t has_fixed;      // some owner is in a fixed family (its flag in AcsBuf::oany, bit 1)
    int32_t two_kernel;     // the step runs as force + fold kernels (one block per 256 owners)
    // a set adopted right before this step whose history has not been
    // carried over yet: the fused step reads the old history of each pair
    // it finds touching from the previous set (rows rm_start / rm_j,
    // history rm_h*), in place of k_remap; rm_start null: no such set.
    // rm_newbuf: the adopted buffer (its overflow stops the step)
    const uint32_t *rm_start, *rm_j;
    const float *rm_hx, *rm_hy, *rm_hz, *rm_hw;
    int32_t rm_newbuf;
    // a work order whose first binning step rides on this step (single-
    // sphere runs without fixed families): from the state it reads, the
    // step also writes each sphere's bin key and candidate record and
    // counts the bins (each sphere's slot in its bin kept), as k_cd_prepare
    // would; wo_keys null: no such order
    Grid wo_grid;
    uint32_t *wo_keys;
    Cand *wo_cand;
    uint32_t *wo_count;
    uint32_t *wo_rank;
    int32_t dense_rows;     // the last contact count read back was at least one per two spheres: the
                            // fused step stages its history writes in LDS (a choice of speed only:
                            // both variants give the same bits)
    int32_t split;          // clump systems without fixed families: run the step as a streaming
                            // kernel over every owner plus a kernel over the set's owners with
                            // contacts (AcsBuf::olist); the same bits as the one-kernel step
    // Pairs provably apart (systems without fixed families: single spheres
    // in the one-kernel step, clumps in the split step).
    // A chain is a run of consecutive steps on one set; its reach D(n) bounds
    // how far any two surfaces can have closed in since the chain began:
    // D(first) = 0, D(n) = D(n-1) + h (2 v(n) + vgeom) + GAP_STEP_SLACK with
    // v(n) the largest sphere speed the step before integrated (for a clump
    // sphere its owner's |v| + |w| arm: the step turns it by h |w|, which
    // moves a sphere at most h |w| arm).  Evaluating
    // a pair, the step writes gk[c] = (its gap - GAP_PAIR_SLACK) + D(n),
    // rounded down; while gk[c] - D(n) > 0 the pair cannot touch, and the
    // step gives it what evaluating it would: no force, zero history.
    // gap: 0 off, 1 the first step of a chain (every pair evaluated, keys
    // written), 2 a later step (pairs skipped by their keys).
    float *gk;
    int32_t gap;
    float *gvs;             // [3][64] speed slots (max squared speed bits, one per 64 B), by step mod 3
    double *gD;             // [2] reach D by step parity
    double vgeom;           // fastest point of any wall or mesh
    float arm;              // largest distance of a template sphere's centre from its owner's (0: none)
    int32_t nt;             // store the streaming step's records non-temporally (stream_nt)
};

struct StepBufs {
    float *aF, *aT;          // per sphere: 3 floats each (SoA: x[Ns], y[Ns], z[Ns])
    float *bF, *bT;          // per contact: 3 floats each (SoA, cap stride)
    float *Fo, *To;          // per owner output of dem_forces (SoA, No stride)
    int64_t cap;
};

// ev0/ev1 (may be null): events stamped by the dispatch itself around the kernel
void launch_force(const DynArgs &a, AcsBuf &cur, StepBufs &sb, DevCounters *ctr, hipStream_t s,
                  hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void launch_fold_integrate(const DynArgs &a, const AcsBuf &cur, StepBufs &sb, DevCounters *ctr,
                           int integrate, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// one fused step (forces of both sides, ordered sums, integration): reads
// a.rec / a.q and cur's history, writes rec_out / q_out and cur's second
// history buffer; the caller swaps both afterwards.  Returns false (and
// launches nothing) for a combination no kernel variant covers: a work
// order's binning on the first step of a newly adopted set, or in a run
// with clumps or fixed families
// Optional event pairs around the two kernels of a split step.
struct SplitTiming {
    hipEvent_t free0, free1, list0, list1;
};
// the step runs as the streaming kernel plus the kernel over the owners with
// contacts (DynArgs::split, for a system and set that allow it)
bool step_is_split(const DynArgs &a, const AcsBuf &cur);
bool launch_step_fused(const DynArgs &a, RecBuf rec_out, double *q_out, const AcsBuf &cur, int64_t cap,
                       DevCounters *ctr, hipStream_t s, const SplitTiming *tm = nullptr);
// an empty one-wave kernel stamped with events (overhead of the stamps)
void launch_noop(hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// max |v|^2 of the last integration into ctr->maxv2[0]
// adaptive schedule: margin of the next detection from the top speed
// (after launch_reduce_max), into ctr->margin
// owners of fixed families: v = w = 0 in `rec`, and both state buffers equal
void launch_fix_owners(RecBuf rec, RecBuf rec_alt, const double *q, double *q_alt, const uint8_t *ofam,
                       const uint8_t *fixed, int64_t n_owners, hipStream_t s);
void launch_adaptive_margin(DevCounters *ctr, double t, double gmag, double cap, double vfloor, hipStream_t s);
void launch_reduce_max(const DynArgs &a, DevCounters *ctr, hipStream_t s);

// Inputs of the learned schedule's decision on the device (k_learned_decide).
struct LearnedArgs {
    double g;           // |gravity|
    double margin;
    double dt;
    double safety;      // factor on the predicted horizon
    double vgeom;       // fastest point of any wall or mesh
    int64_t lam;        // adoption latency (steps)
    int64_t kmax;       // largest interval
    int32_t use_model;  // a network is installed: predict; else the analytic bound
    int32_t moving;     // some wall or mesh moves (its analytic bound caps the prediction)
    int32_t speed_valid;// the top speed of the last integration is meaningful (a step was taken)
    int32_t ahead;      // steps between the state the features see and the work order (0 or 1)
};

// Learned interval (dem_mlp.hip): the features, the network and the
// decision on the device, writing out[0] = the next interval, out[1] = the
// analytic bound, out[2] = the bits of the smallest prediction; the
// snapshot is overwritten by the current state.
void learned_decide(RecBuf rec, SnapRec *snap, const float *ovol, Origin org, Grid fg, float h,
                    float margin, float tau, uint32_t *raw, const float *params, float *pslot, const float *blkmax,
                    int64_t nblk, const LearnedArgs &p, int64_t *out, int64_t No, hipStream_t s);
int64_t learned_slots(int64_t ncell);
void snapshot_write(RecBuf rec, SnapRec *snap, int64_t No, hipStream_t s);
void feature_pipeline(RecBuf rec, const SnapRec *snap, const float *ovol, Origin org, Grid fg, float h,
                      float margin, float tau, uint32_t *raw, uint32_t *flags, uint32_t *pos, uint32_t *partials,
                      uint32_t *cellmap, float *out, uint32_t *cell_ids, int64_t No, hipStream_t s);
// number of slots of the per-block |v|^2 maxima the last step wrote
int64_t speed_slots(const DynArgs &a);

// message of the last failed context-free call on this host thread
const char *free_call_error();
