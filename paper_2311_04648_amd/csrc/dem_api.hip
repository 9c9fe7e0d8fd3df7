// Host side of the DEM library: context, workspace layout inside one
// caller-owned device buffer, the delayed contact-detection schedule on two
// HIP streams (paper Sec. 2.1), and the C ABI declared in include/dem.h.
//
// Schedule (FIXED / LEARNED): a work order at step s copies the owner state
// into a snapshot on the dynamics stream, records an event, and the
// detection stream builds the next active set from the snapshot into the
// buffer not in use.  The dynamics stream adopts it at the deterministic
// step s + lambda (waiting on the detection event only there), remaps the
// contact history from the set in use, and carries on.  Because adoption
// happens at a fixed step, the trajectory does not depend on timing.
#include "dem_device.h"
#include "../../include/dem.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

constexpr int64_t POSE_RING = 512, POSE_CHUNK = 256;

// A host thread that enqueues the detection-stream part of each work order
// (its wait for the work-order event and a dozen launches), so that the
// thread driving the dynamics stream keeps that stream fed meanwhile: the
// paper, too, drives its kinematic and dynamic parts from separate host
// threads (Sec. 2.1).  One job at a time; the dynamics thread waits for the
// job to be enqueued (kin_join) before anything that depends on it.
struct KinWorker {
    std::thread th;
    std::mutex m;
    std::condition_variable cv;
    std::function<void()> job;
    bool busy = false, quit = false;
    hipError_t err = hipSuccess;   // first launch error of a job since the last join
    int device = 0;
};

static void kin_loop(KinWorker *w)
{
    hipSetDevice(w->device);
    std::unique_lock<std::mutex> lk(w->m);
    for (;;) {
        w->cv.wait(lk, [w] { return w->quit || static_cast<bool>(w->job); });
        if (!w->job) return;
        std::function<void()> job = std::move(w->job);
        w->job = nullptr;
        lk.unlock();
        job();
        const hipError_t e = hipGetLastError();
        lk.lock();
        if (e != hipSuccess && w->err == hipSuccess) w->err = e;
        w->busy = false;
        w->cv.notify_all();
    }
}

struct dem_ctx {
    std::string err;
    dem_params P;
    int64_t No = 0, Ns = 0;
    int32_t W = 0, T = 0, nmat = 0, ncomp = 0;
    bool has_clumps = false;
    bool rolling = false;
    std::vector<OwnerAux> aux;
    std::vector<uint32_t> sph0;
    std::vector<SphRec> sph;
    std::vector<float> tpos;
    float arm = 0.0f;   // largest |template position| (rounded up)
    std::vector<WallDev> walls;
    std::vector<MatPair> mat;
    std::vector<float> mass;
    std::vector<int32_t> tmpl;
    double rmax = 0.0;
    // meshes (host copies; poses are evaluated per step on the host)
    int32_t NM = 0, NF = 0;
    std::vector<TriDev> tri;
    std::vector<double> mesh_origin, mesh_vel, mesh_omega;
    std::vector<int32_t> mesh_mat;
    double vmesh = 0.0;          // fastest point of any mesh (m/s)
    double vwall = 0.0;          // fastest point of any wall (m/s)
    TriDev *d_tri = nullptr;
    // mesh poses of the dynamics: a device ring of POSE_RING steps, filled
    // POSE_CHUNK steps at a time from pinned staging (two halves, each reused
    // after its previous copy has completed)
    MeshPose *d_pose_ring = nullptr;    // [POSE_RING * NM]
    MeshPose *h_pose_stage = nullptr;   // pinned [2 * POSE_CHUNK * NM]
    hipEvent_t ev_pose[2] = {nullptr, nullptr};
    int64_t pose_lo = 0, pose_hi = 0;   // steps whose poses the ring holds (the last chunk)
    int pose_half = 0;
    // family tags: per owner, per mesh (walls keep theirs in WallDev), the
    // switched-off family pairs and the fixed families
    std::vector<uint8_t> ofam, mesh_family, pairoff, famfixed, famdormant;
    bool has_pairoff = false, has_fixed = false, has_state = false, has_dormant = false;
    uint8_t *d_ofam = nullptr, *d_pairoff = nullptr, *d_famfixed = nullptr, *d_famdormant = nullptr;
    // static index of the dormant spheres (rebuilt when the tags or the state are set)
    uint32_t *d_dcell_start = nullptr;
    Cand *d_dcand = nullptr;
    float4 *d_dcandf = nullptr;
    Grid grid{};
    Grid fgrid{};
    Origin org{};
    double bin_size = 0.0;
    int sort_bits = 0;
    // binding
    bool bound = false;
    char *ws = nullptr;
    int64_t ws_bytes = 0, cap = 0;
    RecBuf rec{nullptr, nullptr};
    RecBuf rec_alt{nullptr, nullptr};    // the fused step writes here, then the two swap
    double *q_alt = nullptr;
    SnapRec *fref = nullptr;        // reference state of the learned-interval features
    float *d_ovol = nullptr;        // volume of each owner's spheres (packing-fraction feature)
    double *q = nullptr;
    OwnerAux *d_aux = nullptr;
    float *d_inv_i = nullptr;
    uint32_t *d_sph0 = nullptr;
    uint2 *d_sph_range = nullptr;   // [Ns] owner's sphere range of each sphere (clump systems)
    SphRec *d_sph = nullptr;
    float *d_tpos = nullptr;
    WallDev *d_walls = nullptr;
    MatPair *d_mat = nullptr;
    AcsBuf acs[2]{};
    StepBufs sb{};
    CdWork cdK{}, cdD{};
    DevCounters *ctr = nullptr;
    DevCounters *h_ctr = nullptr;
    // pair skipping (single-sphere systems): the speed slots and reaches of
    // the chains, and a count of adoptions (a chain lives on one adopted set)
    float *d_gvs = nullptr;
    double *d_gD = nullptr;
    uint64_t adopt_epoch = 0;
    // learned interval
    float *d_blkmax = nullptr;
    float *d_mlp = nullptr;
    float *d_feat = nullptr, *d_pred = nullptr;
    uint32_t *d_cellmap = nullptr;    // feature cell of each owner [No]
    uint32_t *d_fraw = nullptr;       // raw per-cell accumulators [16 ncell]
    uint32_t *d_fflag = nullptr, *d_fpos = nullptr, *d_fids = nullptr;
    uint32_t *d_lab_start = nullptr, *d_lab_j = nullptr;   // label set (training logs)
    int64_t ncell_cap = 0;
    int64_t snap_step = 0;
    std::vector<float> mlp;
    bool mlp_set = false;
    float *h_pred = nullptr;
    // the learned schedule's decision: device output (interval, analytic
    // bound, smallest prediction), its pinned copy, the per-block prediction
    // minima; a decision enqueued one step ahead of its work order
    int64_t *d_kdec = nullptr;
    int64_t *h_kdec = nullptr;
    float *d_pslot = nullptr;
    hipEvent_t ev_kdec = nullptr;
    bool prep_valid = false;
    int64_t prep_step = -1;
    // schedule
    int64_t step = 0;
    int cur = 0;
    bool sched_init = false;
    bool pending = false;
    int64_t pend_swap = 0, next_wo = 0, last_wo = 0;
    int pend_buf = 1;
    hipEvent_t ev_wo = nullptr, ev_cd = nullptr;
    KinWorker *kw = nullptr;   // started at the first work order on a separate detection stream
    bool cdk_zeroed = false;   // cdK's bin counts hold zeros (each work order's back part leaves them so)
    // a work order whose first binning step rides on the next fused step:
    // what is left to enqueue after that step (the work-order event and the
    // detection-stream part), and what the step needs (wo_args, wo_target)
    bool wo_fused = false;
    std::function<void()> wo_finish;
    DetectArgs wo_args{};
    int wo_target = 0;
    int rm_from = -1;          // set adopted before the next fused step without its history carried over:
                               // the buffer to carry it from (-1: none)
    // adaptive schedule: per work-order cycle, timing events at the work
    // order (dynamics stream), at the end of its detection (detection
    // stream) and at its adoption step before the wait (dynamics stream)
    struct Cycle {
        hipEvent_t wo = nullptr, cd = nullptr, adopt = nullptr;
        int lam = 0;
        bool issued = false, adopted = false;
    };
    Cycle cyc[4];
    int cyc_pos = 0;
    uint32_t *h_capped = nullptr;   // pinned, one flag per cycle slot
    int lam_cur = 1;
    int64_t n_wo = 0;
    double interval_sum = 0.0;
    // stage timing (params.timing): a ring of event pairs, drained lazily
    struct TimedPair {
        hipEvent_t a = nullptr, b = nullptr;
        int kind = -1;
        int count = 1;      // launches between the two events
    };
    TimedPair *run = nullptr;   // open run of timed back-to-back dynamics launches
    int run_len = 0;
    bool run_due = false;       // a sampling mark passed; open a run when possible
    std::vector<TimedPair> ring;
    size_t ring_pos = 0;
    double stage_ms[5] = {0, 0, 0, 0, 0};
    int64_t stage_n[5] = {0, 0, 0, 0, 0};
};

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
            return DEM_ERR_HIP;                                                        \
        }                                                                              \
    } while (0)

#define ARGCHK(cond, msg)                                                              \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            ctx->err = (msg);                                                          \
            return DEM_ERR_ARG;                                                        \
        }                                                                              \
    } while (0)

namespace {

// Carves aligned sub-buffers out of the caller's workspace (base == nullptr:
// only measure).
struct Carver {
    char *base;
    int64_t off = 0;
    explicit Carver(char *b) : base(b) {}
    template <typename T>
    T *take(int64_t n)
    {
        off = (off + 255) & ~int64_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (int64_t)sizeof(T) * std::max<int64_t>(n, 1);
        return p;
    }
};

int64_t partial_elems(const dem_ctx *ctx)
{
    int64_t n = std::max<int64_t>(ctx->Ns + 1, (int64_t)ctx->grid.nbins + 1);
    n = std::max<int64_t>(n, radix_hist_elems(ctx->Ns));
    return 2 * scan_tmp_elems(n) + 16;
}

void carve_cd(Carver &c, const dem_ctx *ctx, CdWork &w)
{
    int64_t ns = ctx->Ns;
    w.keys = c.take<uint32_t>(ns);
    w.vals = c.take<uint32_t>(ns);
    w.keys_alt = c.take<uint32_t>(ns);
    w.vals_alt = c.take<uint32_t>(ns);
    w.rank = c.take<uint32_t>(ns);
    w.cand_tmp = c.take<Cand>(ns);
    w.cand = c.take<Cand>(ns);
    w.candf = c.take<float4>(ns);
    w.cell_count = c.take<uint32_t>((int64_t)ctx->grid.nbins + 1);
    w.cell_start = c.take<uint32_t>((int64_t)ctx->grid.nbins + 1);
    w.count = c.take<uint32_t>(ns + 1);
    w.stage = c.take<uint32_t>(16 * ns);
    w.hist = c.take<uint32_t>(radix_hist_elems(ns));
    w.partials = c.take<uint32_t>(partial_elems(ctx));
    w.fac = c.take<FacetDev>(ctx->NF);
    w.frow = c.take<uint32_t>((int64_t)ctx->NF + 1);
    w.sort_bits = ctx->sort_bits;
    w.sort_mode = ctx->P.bin_sort;
}

void carve(Carver &c, dem_ctx *ctx, int64_t cap)
{
    int64_t No = ctx->No, Ns = ctx->Ns;
    // (clump systems split each record into a hot and a cold part; single-
    // sphere systems keep whole records)
    for (RecBuf *b : {&ctx->rec, &ctx->rec_alt}) {
        b->hot = c.take<uint4>((ctx->has_clumps ? 2 : 3) * No);
        b->cold = ctx->has_clumps ? c.take<uint4>(No) : nullptr;
    }
    ctx->fref = c.take<SnapRec>(No);
    ctx->d_ovol = c.take<float>(No);
    ctx->q = c.take<double>(4 * No);
    ctx->q_alt = c.take<double>(4 * No);
    ctx->d_aux = c.take<OwnerAux>(No);
    ctx->d_inv_i = c.take<float>(No);
    ctx->d_sph0 = c.take<uint32_t>(No + 1);
    ctx->d_sph_range = c.take<uint2>(ctx->has_clumps ? Ns : 0);
    ctx->d_sph = c.take<SphRec>(Ns);
    ctx->d_tpos = c.take<float>(4 * std::max(ctx->ncomp, 1));
    ctx->d_walls = c.take<WallDev>(std::max(ctx->W, 1));
    ctx->d_tri = c.take<TriDev>(ctx->NF);
    ctx->d_ofam = c.take<uint8_t>(No);
    ctx->d_pairoff = c.take<uint8_t>(256 * 256);
    ctx->d_famfixed = c.take<uint8_t>(256);
    ctx->d_famdormant = c.take<uint8_t>(256);
    ctx->d_dcell_start = c.take<uint32_t>((int64_t)ctx->grid.nbins + 1);
    ctx->d_dcand = c.take<Cand>(Ns);
    ctx->d_dcandf = c.take<float4>(Ns);
    ctx->d_pose_ring = c.take<MeshPose>(POSE_RING * ctx->NM);
    ctx->d_mat = c.take<MatPair>((int64_t)ctx->nmat * ctx->nmat);
    for (int b = 0; b < 2; ++b) {
        AcsBuf &a = ctx->acs[b];
        a.start = c.take<uint32_t>(Ns + 1);
        a.j = c.take<uint32_t>(cap);
        a.hx = c.take<float>(cap);
        a.hy = c.take<float>(cap);
        a.hz = c.take<float>(cap);
        a.hw = c.take<float>(cap);
        a.hx2 = c.take<float>(cap);
        a.hy2 = c.take<float>(cap);
        a.hz2 = c.take<float>(cap);
        a.hw2 = c.take<float>(cap);
        a.bstart = c.take<uint32_t>(Ns + 1);
        a.bidx = c.take<uint32_t>(cap);
        a.bsrc = c.take<uint32_t>(cap);
        a.bcur = c.take<uint32_t>(Ns + 1);
        a.oany = c.take<uint8_t>(No);
        a.olist = c.take<uint4>(ctx->has_clumps ? 2 * No : 1);
        a.otile = c.take<uint32_t>(owner_list_tiles(No) + 1);
        a.gk = c.take<float>(cap);
    }
    ctx->d_gvs = c.take<float>(3 * 64 * 16);
    ctx->d_gD = c.take<double>(2);
    ctx->sb.aF = c.take<float>(3 * Ns);
    ctx->sb.aT = c.take<float>(3 * Ns);
    ctx->sb.bF = c.take<float>(3 * cap);
    ctx->sb.bT = c.take<float>(3 * cap);
    ctx->sb.Fo = c.take<float>(3 * No);
    ctx->sb.To = c.take<float>(3 * No);
    ctx->sb.cap = cap;
    ctx->d_blkmax = c.take<float>((No + 255) / 256 + 1);
    carve_cd(c, ctx, ctx->cdK);
    ctx->cdk_zeroed = false;
    carve_cd(c, ctx, ctx->cdD);
    ctx->ctr = c.take<DevCounters>(1);
    ctx->ncell_cap = (int64_t)ctx->fgrid.nbins;
    ctx->d_mlp = c.take<float>(DEM_MLP_NPARAM + 3);
    ctx->d_cellmap = c.take<uint32_t>(No);
    ctx->d_fraw = c.take<uint32_t>(16 * ctx->ncell_cap);
    ctx->d_fflag = c.take<uint32_t>(ctx->ncell_cap + 1);
    ctx->d_fpos = c.take<uint32_t>(ctx->ncell_cap + 1);
    ctx->d_fids = c.take<uint32_t>(ctx->ncell_cap + 1);
    ctx->d_feat = c.take<float>(DEM_MLP_NFEAT * ctx->ncell_cap);
    ctx->d_pred = c.take<float>(ctx->ncell_cap + 4);
    ctx->d_pslot = c.take<float>(learned_slots(ctx->ncell_cap));
    ctx->d_kdec = c.take<int64_t>(4);
    ctx->d_lab_start = c.take<uint32_t>(Ns + 1);
    ctx->d_lab_j = c.take<uint32_t>(cap);
}

// Pose of mesh g at step n (t = n dt): reference point origin + vel t, and
// the rotation by the angle |omega| t about omega / |omega| (Rodrigues'
// formula), in FP64 on the host.
void mesh_pose(const dem_ctx *ctx, int g, int64_t step, MeshPose &P)
{
    const double t = (double)step * ctx->P.dt;
    const double *o = &ctx->mesh_origin[3 * g], *v = &ctx->mesh_vel[3 * g], *w = &ctx->mesh_omega[3 * g];
    for (int k = 0; k < 3; ++k) {
        P.p[k] = o[k] + v[k] * t;
        P.vel[k] = (float)v[k];
        P.omega[k] = (float)w[k];
    }
    P.mat = ctx->mesh_mat[g];
    P.family = ctx->mesh_family.empty() ? 0 : ctx->mesh_family[g];
    const double wn = std::sqrt((w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]);
    if (!(wn > 0.0)) {
        for (int k = 0; k < 9; ++k) P.R[k] = (k % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    const double ux = w[0] / wn, uy = w[1] / wn, uz = w[2] / wn;
    const double ang = wn * t;
    const double c = std::cos(ang), sn = std::sin(ang), C = 1.0 - c;
    P.R[0] = c + ux * ux * C;
    P.R[1] = ux * uy * C - uz * sn;
    P.R[2] = ux * uz * C + uy * sn;
    P.R[3] = uy * ux * C + uz * sn;
    P.R[4] = c + uy * uy * C;
    P.R[5] = uy * uz * C - ux * sn;
    P.R[6] = uz * ux * C - uy * sn;
    P.R[7] = uz * uy * C + ux * sn;
    P.R[8] = c + uz * uz * C;
}

MeshPoses mesh_poses(const dem_ctx *ctx, int64_t step)
{
    MeshPoses M;
    std::memset(&M, 0, sizeof(M));
    for (int g = 0; g < ctx->NM; ++g) mesh_pose(ctx, g, step, M.m[g]);
    return M;
}

// Clump systems without fixed families keep, with every set, the list of
// its owners with contacts (the split step runs over it).
inline bool owner_list_wanted(const dem_ctx *ctx)
{
    return ctx->has_clumps && !ctx->has_fixed && ctx->P.dyn_path != 1;
}

DetectArgs detect_args(const dem_ctx *ctx, double margin, int64_t step)
{
    DetectArgs a;
    a.recs = ctx->rec;
    a.q = ctx->q;
    a.aux = ctx->d_aux;
    a.sph = ctx->d_sph;
    a.tpos = ctx->d_tpos;
    a.walls = ctx->d_walls;
    a.n_walls = ctx->W;
    a.n_spheres = ctx->Ns;
    a.grid = ctx->grid;
    a.org = ctx->org;
    a.margin = margin;
    a.margin_dev = nullptr;
    a.own_sph0 = ctx->has_clumps ? ctx->d_sph0 : nullptr;
    a.sph_range = ctx->has_clumps ? ctx->d_sph_range : nullptr;
    a.n_owners = ctx->No;
    a.h = ctx->P.dt;
    a.step = step;
    a.rmax = ctx->rmax;
    a.tri = ctx->d_tri;
    a.n_tri = ctx->NF;
    a.poses = mesh_poses(ctx, step);
    a.ofam = ctx->d_ofam;
    a.pairoff = ctx->has_pairoff ? ctx->d_pairoff : nullptr;
    a.famfixed = ctx->has_fixed ? ctx->d_famfixed : nullptr;
    a.famdormant = ctx->has_dormant ? ctx->d_famdormant : nullptr;
    a.dcell_start = ctx->d_dcell_start;
    a.dcand = ctx->d_dcand;
    a.dcandf = ctx->d_dcandf;
    a.owner_list = owner_list_wanted(ctx) ? 1 : 0;
    a.nt = stream_nt(ctx->No) ? 1 : 0;
    return a;
}

DynArgs dyn_args(const dem_ctx *ctx, int64_t step)
{
    DynArgs a;
    a.recs = ctx->rec;
    a.q = ctx->q;
    a.aux = ctx->d_aux;
    a.inv_i = ctx->d_inv_i;
    a.own_sph0 = ctx->d_sph0;
    a.sph = ctx->d_sph;
    a.tpos = ctx->d_tpos;
    a.walls = ctx->d_walls;
    a.mat = ctx->d_mat;
    a.n_mat = ctx->nmat;
    a.n_walls = ctx->W;
    a.n_owners = ctx->No;
    a.n_spheres = ctx->Ns;
    a.org = ctx->org;
    a.h = ctx->P.dt;
    for (int k = 0; k < 3; ++k) a.g[k] = (float)ctx->P.gravity[k];
    a.v_err2 = (float)(ctx->P.v_error_out * ctx->P.v_error_out);
    a.step = step;
    a.has_clumps = ctx->has_clumps ? 1 : 0;
    a.rolling = ctx->rolling ? 1 : 0;
    a.cur = ctx->cur;
    a.blkmax = ctx->d_blkmax;
    a.tri = ctx->d_tri;
    a.n_tri = ctx->NF;
    a.poses = nullptr;
    a.has_fixed = ctx->has_fixed ? 1 : 0;
    a.two_kernel = ctx->P.dyn_path == 1 ? 1 : 0;
    a.rm_start = a.rm_j = nullptr;
    a.rm_hx = a.rm_hy = a.rm_hz = a.rm_hw = nullptr;
    a.rm_newbuf = ctx->cur;
    if (ctx->rm_from >= 0) {
        const AcsBuf &o = ctx->acs[ctx->rm_from];
        a.rm_start = o.start;
        a.rm_j = o.j;
        a.rm_hx = o.hx;
        a.rm_hy = o.hy;
        a.rm_hz = o.hz;
        a.rm_hw = o.hw;
    }
    a.wo_grid = ctx->grid;
    a.wo_keys = nullptr;
    a.wo_cand = nullptr;
    a.wo_count = nullptr;
    a.wo_rank = nullptr;
    if (ctx->wo_fused) {
        a.wo_keys = ctx->cdK.keys;
        a.wo_cand = ctx->cdK.cand_tmp;
        a.wo_count = ctx->cdK.cell_count;
        a.wo_rank = ctx->cdK.rank;
    }
    a.dense_rows = 0;
    if (ctx->P.dyn_path == 2) {
        a.dense_rows = 1;
    } else if (ctx->P.dyn_path == 0 && ctx->h_ctr) {
        const int64_t nc = std::max(ctx->h_ctr->n_contacts[0], ctx->h_ctr->n_contacts[1]);
        a.dense_rows = 2 * nc >= ctx->Ns ? 1 : 0;
    }
    // clump systems without fixed families: a sparse set runs as the
    // streaming kernel plus the kernel over the owners with contacts
    a.split = owner_list_wanted(ctx) && (ctx->P.dyn_path == 4 || (ctx->P.dyn_path == 0 && !a.dense_rows)) ? 1 : 0;
    // pair skipping: off unless dem_step opens or continues a chain
    a.gk = ctx->acs[ctx->cur].gk;
    a.gap = 0;
    a.gvs = ctx->d_gvs;
    a.gD = ctx->d_gD;
    a.vgeom = std::max(ctx->vmesh, ctx->vwall);
    a.arm = ctx->arm;
    a.nt = stream_nt(ctx->No) ? 1 : 0;
    return a;
}

// Systems without fixed families skip the pairs proven apart: single
// spheres in the one-kernel step over a dense set (its staged variant),
// clumps in the split step
static bool pair_skip_allowed(const dem_ctx *ctx, const DynArgs &a)
{
    return !ctx->P.no_pair_skip && !ctx->has_clumps && !ctx->has_fixed && a.dense_rows && a.gk &&
           ctx->P.dyn_path != 1;
}

static bool pair_skip_split_allowed(const dem_ctx *ctx, const DynArgs &a)
{
    return !ctx->P.no_pair_skip && ctx->has_clumps && !ctx->has_fixed && a.gk;
}

inline hipStream_t S(dem_stream s) { return reinterpret_cast<hipStream_t>(s); }

// Device address of the mesh poses of step n, for dynamics kernels enqueued
// on stream s after this call.  A step outside the last chunk refills the
// ring with the POSE_CHUNK steps from n on: poses computed on the host into
// a staging half, copied to ring slots (n + i) mod POSE_RING on s (so after
// every earlier kernel on s that read those slots).  Null without meshes.
const MeshPose *dyn_poses(dem_ctx *ctx, int64_t n, hipStream_t s)
{
    const int64_t nm = ctx->NM;
    if (nm == 0) return nullptr;
    if (!(n >= ctx->pose_lo && n < ctx->pose_hi)) {
        const int h = ctx->pose_half;
        ctx->pose_half ^= 1;
        hipEventSynchronize(ctx->ev_pose[h]);
        MeshPose *st = ctx->h_pose_stage + (size_t)h * POSE_CHUNK * nm;
        for (int64_t i = 0; i < POSE_CHUNK; ++i)
            for (int g = 0; g < (int)nm; ++g) mesh_pose(ctx, g, n + i, st[i * nm + g]);
        const int64_t slot = ((n % POSE_RING) + POSE_RING) % POSE_RING;
        const int64_t first = std::min<int64_t>(POSE_CHUNK, POSE_RING - slot);
        hipMemcpyAsync(ctx->d_pose_ring + slot * nm, st, sizeof(MeshPose) * first * nm, hipMemcpyHostToDevice, s);
        if (first < POSE_CHUNK)
            hipMemcpyAsync(ctx->d_pose_ring, st + first * nm, sizeof(MeshPose) * (POSE_CHUNK - first) * nm,
                           hipMemcpyHostToDevice, s);
        hipEventRecord(ctx->ev_pose[h], s);
        ctx->pose_lo = n;
        ctx->pose_hi = n + POSE_CHUNK;
    }
    const int64_t slot = ((n % POSE_RING) + POSE_RING) % POSE_RING;
    return ctx->d_pose_ring + slot * nm;
}

dem_status read_counters(dem_ctx *ctx, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(ctx->h_ctr, ctx->ctr, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return DEM_OK;
}

void host_rot(const double *q, double *R)
{
    Mat3d M = rot_from_q(q[0], q[1], q[2], q[3]);
    for (int k = 0; k < 9; ++k) R[k] = M.m[k];
}

// Empty active set in buffer b (all rows empty, no B lists).
void clear_set(dem_ctx *ctx, int b, hipStream_t s)
{
    launch_fill_u32(ctx->acs[b].start, ctx->Ns + 1, 0u, s);
    launch_fill_u32(ctx->acs[b].bstart, ctx->Ns + 1, 0u, s);
    launch_owner_flags(ctx->acs[b], ctx->has_clumps ? ctx->d_sph0 : nullptr, ctx->No, ctx->Ns, ctx->cap, ctx->d_ofam,
                       ctx->has_fixed ? ctx->d_famfixed : nullptr, s, owner_list_wanted(ctx), ctx->cdD.partials);
}

void drain_pair(dem_ctx *ctx, dem_ctx::TimedPair &p)
{
    if (p.kind < 0) return;
    float ms = 0.0f;
    hipEventSynchronize(p.b);
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        ctx->stage_ms[p.kind] += ms;
        ctx->stage_n[p.kind] += p.count;
    }
    p.kind = -1;
    p.count = 1;
}

// Opens a timed stage on stream s; returns the pair to close (or null).
// A free event pair for a timed stage (or null when not timing).  Per-step
// kernels are sampled every `timing` steps; detection chains always.
dem_ctx::TimedPair *stage_slot(dem_ctx *ctx, int kind)
{
    if (ctx->P.timing <= 0) return nullptr;
    if ((kind <= 1 || kind == 4) && kind != 5 && (ctx->step % ctx->P.timing) != 0) return nullptr;
    if (kind == 5) kind = 1;   // a run of fused dynamics launches (opened by the caller's own rule)
    if (ctx->ring.empty()) ctx->ring.resize(1024);
    dem_ctx::TimedPair &p = ctx->ring[ctx->ring_pos];
    ctx->ring_pos = (ctx->ring_pos + 1) % ctx->ring.size();
    drain_pair(ctx, p);
    if (!p.a) {
        // no system-scope release at the stamps: they must not add a cache
        // write-back to the kernel they bracket
        hipEventCreateWithFlags(&p.a, hipEventDisableSystemFence);
        hipEventCreateWithFlags(&p.b, hipEventDisableSystemFence);
    }
    p.kind = kind;
    return &p;
}

// Opens a timed chain of kernels on stream s (events recorded around it).
dem_ctx::TimedPair *stage_begin(dem_ctx *ctx, int kind, hipStream_t s)
{
    dem_ctx::TimedPair *p = stage_slot(ctx, kind);
    if (p) hipEventRecord(p->a, s);
    return p;
}

void stage_end(dem_ctx::TimedPair *p, hipStream_t s)
{
    if (p) hipEventRecord(p->b, s);
}

// Runs of RUN_LAUNCHES back-to-back fused dynamics launches are timed with
// one pair of marker events (their overhead is paid once per run and
// measured by an empty kernel bracketed the same way right after the run).
// After each sampling mark (every `timing` steps) a run opens at the first
// step followed by RUN_LAUNCHES - 1 steps with no other dynamics-stream work,
// so runs cover whole quiet stretches of the schedule and sample its phases
// evenly.  With detection on the dynamics stream every step (every-step or
// judged runs) a run is the one launch of a sampled step.  A run is closed
// before any other work is enqueued on the dynamics stream.
constexpr int RUN_LAUNCHES = 4;

void run_close(dem_ctx *ctx, hipStream_t s)
{
    if (!ctx->run) return;
    ctx->run->count = ctx->run_len;
    stage_end(ctx->run, s);
    ctx->run = nullptr;
    ctx->run_len = 0;
    if (auto *tn = stage_slot(ctx, 5)) {
        tn->kind = 4;
        hipEventRecord(tn->a, s);
        launch_noop(s, nullptr, nullptr);
        hipEventRecord(tn->b, s);
    }
}

void drain_all(dem_ctx *ctx)
{
    for (auto &p : ctx->ring) drain_pair(ctx, p);
}

// Hands a job to the detection-stream thread (started on first use, with
// the caller's current device).  The previous job must have been joined.
void kin_post(dem_ctx *ctx, std::function<void()> job)
{
    if (!ctx->kw) {
        ctx->kw = new KinWorker;
        hipGetDevice(&ctx->kw->device);
        ctx->kw->th = std::thread(kin_loop, ctx->kw);
    }
    std::lock_guard<std::mutex> lk(ctx->kw->m);
    ctx->kw->job = std::move(job);
    ctx->kw->busy = true;
    ctx->kw->cv.notify_all();
}

// Waits until the posted job, if any, has been enqueued; returns the first
// launch error of the jobs since the last join.
hipError_t kin_join(dem_ctx *ctx)
{
    if (!ctx->kw) return hipSuccess;
    std::unique_lock<std::mutex> lk(ctx->kw->m);
    ctx->kw->cv.wait(lk, [ctx] { return !ctx->kw->busy; });
    const hipError_t e = ctx->kw->err;
    ctx->kw->err = hipSuccess;
    return e;
}

void kin_stop(dem_ctx *ctx)
{
    if (!ctx->kw) return;
    kin_join(ctx);
    {
        std::lock_guard<std::mutex> lk(ctx->kw->m);
        ctx->kw->quit = true;
        ctx->kw->cv.notify_all();
    }
    ctx->kw->th.join();
    delete ctx->kw;
    ctx->kw = nullptr;
}


}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *dem_last_error(const dem_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : free_call_error();
}

dem_status dem_create(const dem_params *params, const dem_materials *mats, const dem_templates *tmpls,
                      const dem_walls *walls, const dem_bodies *bodies, dem_ctx **out)
{
    if (!out) return DEM_ERR_ARG;
    *out = nullptr;
    dem_ctx *ctx = new dem_ctx();
    auto fail = [&](const std::string &m) {
        ctx->err = m;
        *out = ctx;   // hand the context back so the caller can read the message
        return DEM_ERR_ARG;
    };
    if (!params || !mats || !bodies) return fail("params, materials and bodies are required");
    ctx->P = *params;
    const dem_params &P = ctx->P;
    if (!(P.dt > 0.0)) return fail("dt must be positive");
    if (!(P.margin >= 0.0)) return fail("margin must be >= 0");
    if (P.cd_mode < 0 || P.cd_mode > 3) return fail("unknown cd_mode");
    if (P.cd_mode == DEM_CD_ADAPTIVE && (P.cd_latency < 1 || P.cd_interval_max < 1))
        return fail("the adaptive schedule needs cd_latency >= 1 and cd_interval_max >= 1");
    if (P.dyn_path < 0 || P.dyn_path > 4)
        return fail("dyn_path must be 0 (automatic), 1 (two kernels), 2 or 3 (one fused kernel, history staged "
                    "or not) or 4 (streaming kernel + kernel over the owners with contacts)");
    if (P.bin_sort < 0 || P.bin_sort > 1) return fail("bin_sort must be 0 (one pass) or 1 (radix)");
    if (P.cd_mode != DEM_CD_EVERY) {
        if (P.cd_interval < 1) return fail("cd_interval must be >= 1");
        if (P.cd_latency < 0 || P.cd_latency > P.cd_interval) return fail("need 0 <= cd_latency <= cd_interval");
    }
    if (P.cd_interval_max < 1) ctx->P.cd_interval_max = std::max(P.cd_interval, 1) * 16;
    ctx->No = bodies->n_owners;
    ctx->Ns = bodies->n_spheres;
    if (ctx->No < 1 || ctx->Ns < ctx->No) return fail("need n_spheres >= n_owners >= 1");
    if (ctx->Ns >= (int64_t)0xffffff00) return fail("too many spheres for 32-bit ids");
    ctx->nmat = mats->n;
    if (ctx->nmat < 1 || ctx->nmat > 256) return fail("material count must be 1..256");
    ctx->W = walls ? walls->n : 0;
    ctx->T = tmpls ? tmpls->n : 0;
    // materials: pairwise constants of Sec. 4.2.1 (E*, G*, beta, mu)
    for (int a = 0; a < ctx->nmat; ++a) {
        if (!(mats->E[a] > 0.0) || !(mats->nu[a] > -1.0 && mats->nu[a] < 0.5))
            return fail("material E must be > 0 and -1 < nu < 0.5");
    }
    ctx->mat.resize((size_t)ctx->nmat * ctx->nmat);
    for (int a = 0; a < ctx->nmat; ++a)
        for (int b = 0; b < ctx->nmat; ++b) {
            double Ea = mats->E[a], na = mats->nu[a], Eb = mats->E[b], nb = mats->nu[b];
            double Es = 1.0 / ((1.0 - na * na) / Ea + (1.0 - nb * nb) / Eb);
            double Gs = 1.0 / (2.0 * (2.0 - na) * (1.0 + na) / Ea + 2.0 * (2.0 - nb) * (1.0 + nb) / Eb);
            double cor = mats->cor[a * ctx->nmat + b];
            double le = (cor < 1e-12) ? std::log(1e-12) : std::log(cor);
            double beta = le / std::sqrt(le * le + M_PI * M_PI);
            MatPair mp;
            mp.Estar = (float)Es;
            mp.Gstar = (float)Gs;
            mp.beta = (float)beta;
            mp.mu = (float)mats->mu[a * ctx->nmat + b];
            double crr = mats->crr ? mats->crr[a * ctx->nmat + b] : 0.0;
            if (!(crr >= 0.0)) return fail("rolling-resistance coefficients must be >= 0");
            mp.crr = (float)crr;
            mp.kns = 0.0f;
            mp.tcol = 0.0f;
            mp.pad = 0.0f;
            if (crr > 0.0) ctx->rolling = true;
            ctx->mat[(size_t)a * ctx->nmat + b] = mp;
        }
    // templates
    std::vector<int32_t> tb(ctx->T + 1, 0);
    if (ctx->T > 0) {
        for (int t = 0; t <= ctx->T; ++t) tb[t] = tmpls->sph_begin[t];
        ctx->ncomp = tb[ctx->T];
        ctx->tpos.resize(4 * (size_t)std::max(ctx->ncomp, 1), 0.0f);
        for (int k = 0; k < ctx->ncomp; ++k)
            for (int d = 0; d < 3; ++d) {
                double v = tmpls->sph_pos[3 * k + d];
                float f = (float)v;
                if ((double)f != v) return fail("template positions must be float32-representable");
                ctx->tpos[4 * k + d] = f;
            }
        // (FP64 norms of FP32 positions, rounded up to FP32)
        double am = 0.0;
        for (int k = 0; k < ctx->ncomp; ++k) {
            const double x = ctx->tpos[4 * k], y = ctx->tpos[4 * k + 1], z = ctx->tpos[4 * k + 2];
            am = std::max(am, std::sqrt(x * x + y * y + z * z));
        }
        float af = (float)am;
        if ((double)af < am) af = std::nextafter(af, 1.0f);
        ctx->arm = af;
    } else {
        ctx->tpos.assign(4, 0.0f);
    }
    // owners and spheres
    ctx->aux.resize(ctx->No);
    ctx->sph0.resize(ctx->No + 1);
    ctx->mass.resize(ctx->No);
    ctx->tmpl.resize(ctx->No);
    ctx->sph.resize(ctx->Ns);
    for (int64_t o = 0; o <= ctx->No; ++o) ctx->sph0[o] = (uint32_t)bodies->own_sph0[o];
    if (ctx->sph0[0] != 0 || (int64_t)ctx->sph0[ctx->No] != ctx->Ns) return fail("own_sph0 must span all spheres");
    for (int64_t o = 0; o < ctx->No; ++o) {
        int32_t t = bodies->own_tmpl[o];
        uint32_t s0 = ctx->sph0[o], s1 = ctx->sph0[o + 1];
        if (s1 <= s0) return fail("every owner needs at least one sphere");
        if (t >= ctx->T) return fail("owner template index out of range");
        if (t < 0 && s1 - s0 != 1) return fail("a single-sphere owner must have exactly one sphere");
        if (t >= 0 && (int)(s1 - s0) != tb[t + 1] - tb[t]) return fail("owner sphere count differs from its template");
        if (t >= 0) ctx->has_clumps = true;
        double m = bodies->own_mass[o];
        if (!(m > 0.0)) return fail("owner mass must be positive");
        ctx->mass[o] = (float)m;
        ctx->tmpl[o] = t;
        OwnerAux a;
        for (int d = 0; d < 3; ++d) {
            double I = bodies->own_moi[3 * o + d];
            if (!(I > 0.0)) return fail("owner inertia must be positive");
            a.inv_moi[d] = (float)(1.0 / (double)(float)I);
        }
        if (t < 0) {
            a.inv_moi[1] = a.inv_moi[0];
            a.inv_moi[2] = a.inv_moi[0];
        }
        a.tmpl = t;
        ctx->aux[o] = a;
        for (uint32_t s = s0; s < s1; ++s) {
            SphRec r;
            r.owner = (uint32_t)o;
            double rad = bodies->sph_rad[s];
            if (!(rad > 0.0)) return fail("sphere radius must be positive");
            r.rad = (float)rad;
            int32_t mt = bodies->sph_mat[s];
            if (mt < 0 || mt >= ctx->nmat) return fail("sphere material out of range");
            r.mat = (uint32_t)mt;
            if (t < 0) {
                r.tcomp = DEM_NO_COMP;
            } else {
                int32_t comp = bodies->sph_comp[s];
                if (comp < 0 || comp >= tb[t + 1] - tb[t]) return fail("sphere component out of range");
                r.tcomp = (uint32_t)(tb[t] + comp);
            }
            ctx->sph[s] = r;
            ctx->rmax = std::max(ctx->rmax, rad);
        }
    }
    // walls
    ctx->walls.resize(std::max(ctx->W, 1));
    for (int w = 0; w < ctx->W; ++w) {
        WallDev d{};
        d.type = walls->type[w];
        if (d.type != DEM_WALL_PLANE && d.type != DEM_WALL_CYLINDER) return fail("unknown wall type");
        for (int k = 0; k < 8; ++k) d.geom[k] = walls->geom[8 * w + k];
        for (int k = 0; k < 3; ++k) {
            d.vel[k] = walls->vel ? walls->vel[3 * w + k] : 0.0;
            d.omega[k] = walls->omega ? walls->omega[3 * w + k] : 0.0;
        }
        d.mat = walls->mat[w];
        if (d.mat < 0 || d.mat >= ctx->nmat) return fail("wall material out of range");
        ctx->walls[w] = d;
        // how fast the wall's surface moves: walls only translate (omega sets
        // the surface velocity of a cylinder, not its shape's motion)
        ctx->vwall = std::max(ctx->vwall, std::sqrt(d.vel[0] * d.vel[0] + d.vel[1] * d.vel[1] +
                                                    d.vel[2] * d.vel[2]));
    }
    // bins: edge >= 2 (r_max + m) with a small safety factor
    double b = 2.0 * (ctx->rmax + P.margin) * (1.0 + 1e-6) + 1e-12;
    ctx->bin_size = b;
    uint64_t nb = 1;
    int dims[3];
    for (int k = 0; k < 3; ++k) {
        double lo = P.domain_lo[k] - b, hi = P.domain_hi[k] + b;
        if (!(hi > lo)) return fail("domain_hi must exceed domain_lo");
        int64_t nint = (int64_t)std::ceil((hi - lo) / b);
        if (nint < 1) nint = 1;
        dims[k] = (int)std::min<int64_t>(nint + 2, 1 << 30);
        ctx->grid.lo[k] = lo;
        nb *= (uint64_t)dims[k];
    }
    if (nb >= 0xfffffff0ull) return fail("domain too large for the bin grid (more than 2^32 bins)");
    ctx->grid.nx = dims[0];
    ctx->grid.ny = dims[1];
    ctx->grid.nz = dims[2];
    ctx->grid.nbins = (uint32_t)nb;
    ctx->grid.inv_b = 1.0 / b;
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= nb) ++bits;   // keys 0 .. nb (nb: a sphere left out of the bins)
    ctx->sort_bits = bits;
    // feature cells of the learned interval: cubes of edge E = 8 (r_max + m)
    // (four times the smallest bin edge) tiling the domain box from its low
    // corner, n_k = ceil(extent_k / E) per axis; a centre outside the box
    // belongs to the nearest cell
    {
        double E = 8.0 * (ctx->rmax + P.margin);
        if (!(E > 0.0)) E = 1.0;
        uint64_t fn = 1;
        int fd[3];
        for (int k = 0; k < 3; ++k) {
            const double c = std::ceil((P.domain_hi[k] - P.domain_lo[k]) / E);
            fd[k] = (int)std::min(std::max(c, 1.0), 1.0e6);
            fn *= (uint64_t)fd[k];
            ctx->fgrid.lo[k] = P.domain_lo[k];
        }
        if (fn >= 0xfffffff0ull) return fail("domain too large for the feature cells");
        ctx->fgrid.nx = fd[0];
        ctx->fgrid.ny = fd[1];
        ctx->fgrid.nz = fd[2];
        ctx->fgrid.nbins = (uint32_t)fn;
        ctx->fgrid.inv_b = 1.0 / E;
    }
    // voxel origin: a multiple of the voxel edge below the grid
    for (int k = 0; k < 3; ++k) {
        double o = std::floor((ctx->grid.lo[k] - b) * DEM_VOXEL_INV) * DEM_VOXEL_SIZE;
        ctx->org.o[k] = o;
        if (P.domain_hi[k] + 2 * b - o >= 127.0) return fail("domain extent must stay below 127 m");
    }
    *out = ctx;
    return DEM_OK;
}

dem_status dem_set_meshes(dem_ctx *ctx, const dem_meshes *meshes)
{
    if (!ctx) return DEM_ERR_ARG;
    if (ctx->bound) {
        ctx->err = "dem_set_meshes after dem_bind (the workspace holds per-facet buffers)";
        return DEM_ERR_STATE;
    }
    const int32_t nm = meshes ? meshes->n_mesh : 0;
    const int64_t nf = meshes && nm > 0 ? meshes->n_tri : 0;
    ARGCHK(nm >= 0 && nm <= DEM_MAX_MESHES, "n_mesh must be 0..DEM_MAX_MESHES");
    ARGCHK(nf >= 0, "n_tri must be >= 0");
    ARGCHK(ctx->Ns + ctx->W + nf < (int64_t)0xfffffff0, "too many geometries for 32-bit partner ids");
    // the facet walk numbers (facet, bin row) pairs with 32-bit integers
    ARGCHK((uint64_t)nf * (uint64_t)ctx->grid.ny * (uint64_t)ctx->grid.nz < 0x7fffffffull,
           "too many facets for the bin grid");
    std::vector<TriDev> tri((size_t)nf);
    std::vector<double> org(3 * (size_t)nm), vel(3 * (size_t)nm), om(3 * (size_t)nm);
    std::vector<int32_t> mat((size_t)nm);
    if (nm > 0) {
        ARGCHK(meshes->origin && meshes->vel && meshes->omega && meshes->mat, "mesh origin, vel, omega, mat are required");
        ARGCHK(nf == 0 || (meshes->tri_mesh && meshes->tri_local), "tri_mesh and tri_local are required");
    }
    for (int32_t g = 0; g < nm; ++g) {
        for (int k = 0; k < 3; ++k) {
            org[3 * g + k] = meshes->origin[3 * g + k];
            vel[3 * g + k] = meshes->vel[3 * g + k];
            om[3 * g + k] = meshes->omega[3 * g + k];
            ARGCHK(std::isfinite(org[3 * g + k]) && std::isfinite(vel[3 * g + k]) && std::isfinite(om[3 * g + k]),
                   "mesh origin, vel and omega must be finite");
        }
        mat[g] = meshes->mat[g];
        ARGCHK(mat[g] >= 0 && mat[g] < ctx->nmat, "mesh material out of range");
    }
    std::vector<double> reach((size_t)nm, 0.0);   // largest vertex distance from the reference point
    for (int64_t f = 0; f < nf; ++f) {
        TriDev t{};
        t.mesh = meshes->tri_mesh[f];
        ARGCHK(t.mesh >= 0 && t.mesh < nm, "facet of an unknown mesh");
        for (int k = 0; k < 9; ++k) {
            t.v[k] = meshes->tri_local[9 * f + k];
            ARGCHK(std::isfinite(t.v[k]), "facet vertices must be finite");
        }
        for (int v = 0; v < 3; ++v) {
            const double *x = t.v + 3 * v;
            reach[t.mesh] = std::max(reach[t.mesh], std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
        }
        tri[(size_t)f] = t;
    }
    double vm = 0.0;
    for (int32_t g = 0; g < nm; ++g) {
        const double *v = &vel[3 * g], *w = &om[3 * g];
        vm = std::max(vm, std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) +
                              std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]) * reach[g]);
    }
    ctx->NM = nm;
    ctx->NF = (int32_t)nf;
    ctx->tri.swap(tri);
    ctx->mesh_origin.swap(org);
    ctx->mesh_vel.swap(vel);
    ctx->mesh_omega.swap(om);
    ctx->mesh_mat.swap(mat);
    ctx->vmesh = vm;
    return DEM_OK;
}

dem_status dem_workspace_size(const dem_ctx *cctx, int64_t contact_capacity, int64_t *bytes)
{
    dem_ctx *ctx = const_cast<dem_ctx *>(cctx);
    if (!ctx || !bytes) return DEM_ERR_ARG;
    ARGCHK(contact_capacity >= 1 && contact_capacity < (int64_t)0xfffffff0, "contact capacity must be 1..2^32-16");
    dem_ctx tmp = *ctx;
    Carver c(nullptr);
    carve(c, &tmp, contact_capacity);
    *bytes = c.off + 256;
    return DEM_OK;
}

dem_status dem_bind(dem_ctx *ctx, void *device_workspace, int64_t bytes, int64_t contact_capacity)
{
    if (!ctx) return DEM_ERR_ARG;
    int64_t need = 0;
    dem_status st = dem_workspace_size(ctx, contact_capacity, &need);
    if (st != DEM_OK) return st;
    ARGCHK(device_workspace != nullptr, "workspace pointer is NULL");
    ARGCHK(((uintptr_t)device_workspace & 255) == 0, "workspace must be 256-byte aligned");
    ARGCHK(bytes >= need, "workspace smaller than dem_workspace_size");
    ctx->ws = reinterpret_cast<char *>(device_workspace);
    ctx->ws_bytes = bytes;
    ctx->cap = contact_capacity;
    Carver c(ctx->ws);
    carve(c, ctx, contact_capacity);
    if (!ctx->h_ctr) {
        HIPCHK(hipHostMalloc((void **)&ctx->h_ctr, sizeof(DevCounters)));
        memset(ctx->h_ctr, 0, sizeof(DevCounters));
    }
    if (!ctx->h_pred) HIPCHK(hipHostMalloc((void **)&ctx->h_pred, 64));
    if (!ctx->h_kdec) HIPCHK(hipHostMalloc((void **)&ctx->h_kdec, 4 * sizeof(int64_t)));
    if (!ctx->ev_kdec) HIPCHK(hipEventCreateWithFlags(&ctx->ev_kdec, hipEventDisableTiming));
    ctx->prep_valid = false;
    // (the work-order events order two streams of one device: no
    // system-scope release is needed at their records)
    if (!ctx->ev_wo) HIPCHK(hipEventCreateWithFlags(&ctx->ev_wo, hipEventDisableTiming | hipEventDisableSystemFence));
    if (!ctx->ev_cd) HIPCHK(hipEventCreateWithFlags(&ctx->ev_cd, hipEventDisableTiming | hipEventDisableSystemFence));
    if (!ctx->h_capped) HIPCHK(hipHostMalloc((void **)&ctx->h_capped, 4 * sizeof(uint32_t)));
    if (ctx->NM > 0) {
        if (ctx->h_pose_stage) HIPCHK(hipHostFree(ctx->h_pose_stage));
        ctx->h_pose_stage = nullptr;
        HIPCHK(hipHostMalloc((void **)&ctx->h_pose_stage, sizeof(MeshPose) * 2 * POSE_CHUNK * ctx->NM));
        for (auto &e : ctx->ev_pose)
            if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    ctx->pose_lo = ctx->pose_hi = 0;
    for (auto &c : ctx->cyc) {
        if (!c.wo) HIPCHK(hipEventCreate(&c.wo));
        if (!c.cd) HIPCHK(hipEventCreate(&c.cd));
        if (!c.adopt) HIPCHK(hipEventCreate(&c.adopt));
    }
    HIPCHK(hipMemcpy(ctx->d_aux, ctx->aux.data(), sizeof(OwnerAux) * ctx->No, hipMemcpyHostToDevice));
    {
        std::vector<float> inv_i(ctx->No);
        for (int64_t o = 0; o < ctx->No; ++o) inv_i[o] = ctx->aux[o].inv_moi[0];
        HIPCHK(hipMemcpy(ctx->d_inv_i, inv_i.data(), sizeof(float) * ctx->No, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(ctx->d_sph0, ctx->sph0.data(), sizeof(uint32_t) * (ctx->No + 1), hipMemcpyHostToDevice));
    if (ctx->has_clumps) {
        std::vector<uint2> rng(ctx->Ns);
        for (int64_t o = 0; o < ctx->No; ++o)
            for (uint32_t q = ctx->sph0[o]; q < ctx->sph0[o + 1]; ++q) rng[q] = make_uint2(ctx->sph0[o], ctx->sph0[o + 1]);
        HIPCHK(hipMemcpy(ctx->d_sph_range, rng.data(), sizeof(uint2) * ctx->Ns, hipMemcpyHostToDevice));
    }
    {
        // volume of each owner's spheres, 4/3 pi r^3 summed in FP64 (overlaps
        // of a clump's spheres counted twice), stored as float
        std::vector<float> vol(ctx->No);
        for (int64_t o = 0; o < ctx->No; ++o) {
            double v = 0.0;
            for (uint32_t q = ctx->sph0[o]; q < ctx->sph0[o + 1]; ++q) {
                const double r = (double)ctx->sph[q].rad;
                v += 4.18879020478639098 * r * r * r;
            }
            vol[o] = (float)v;
        }
        HIPCHK(hipMemcpy(ctx->d_ovol, vol.data(), sizeof(float) * ctx->No, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(ctx->d_sph, ctx->sph.data(), sizeof(SphRec) * ctx->Ns, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_tpos, ctx->tpos.data(), sizeof(float) * ctx->tpos.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_walls, ctx->walls.data(), sizeof(WallDev) * ctx->walls.size(), hipMemcpyHostToDevice));
    if (ctx->NF > 0)
        HIPCHK(hipMemcpy(ctx->d_tri, ctx->tri.data(), sizeof(TriDev) * ctx->NF, hipMemcpyHostToDevice));
    if (ctx->ofam.size() != (size_t)ctx->No) ctx->ofam.assign(ctx->No, 0);
    if (ctx->pairoff.size() != 65536) ctx->pairoff.assign(65536, 0);
    if (ctx->famfixed.size() != 256) ctx->famfixed.assign(256, 0);
    HIPCHK(hipMemcpy(ctx->d_ofam, ctx->ofam.data(), ctx->No, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_pairoff, ctx->pairoff.data(), 65536, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(ctx->d_famfixed, ctx->famfixed.data(), 256, hipMemcpyHostToDevice));
    if (ctx->famdormant.size() != 256) ctx->famdormant.assign(256, 0);
    HIPCHK(hipMemcpy(ctx->d_famdormant, ctx->famdormant.data(), 256, hipMemcpyHostToDevice));
    ctx->has_state = false;
    HIPCHK(hipMemcpy(ctx->d_mat, ctx->mat.data(), sizeof(MatPair) * ctx->mat.size(), hipMemcpyHostToDevice));
    DevCounters z{};
    HIPCHK(hipMemcpy(ctx->ctr, &z, sizeof(DevCounters), hipMemcpyHostToDevice));
    launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->d_gvs), 3 * 64 * 16, 0u, nullptr);
    launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->d_gD), 4, 0u, nullptr);
    if (ctx->mlp_set)
        HIPCHK(hipMemcpy(ctx->d_mlp, ctx->mlp.data(), sizeof(float) * DEM_MLP_NPARAM, hipMemcpyHostToDevice));
    clear_set(ctx, 0, nullptr);
    clear_set(ctx, 1, nullptr);
    HIPCHK(hipDeviceSynchronize());
    ctx->cur = 0;
    ctx->sched_init = false;
    ctx->prep_valid = false;
    ctx->pending = false;
    ctx->bound = true;
    return DEM_OK;
}

static void rebuild_dormant_index(dem_ctx *ctx, hipStream_t s);

// Owner records to and from their device form (RecBuf): split, bytes 0-31
// of an OwnerRec are its hot part (two uint4 of the hot array), bytes 32-47
// its cold part; whole records are the OwnerRec bytes themselves.
static dem_status rec_upload(dem_ctx *ctx, const RecBuf &b, const std::vector<OwnerRec> &rec, hipStream_t s)
{
    const size_t n = rec.size();
    if (!b.cold) {
        HIPCHK(hipMemcpyAsync(b.hot, rec.data(), sizeof(OwnerRec) * n, hipMemcpyHostToDevice, s));
        return DEM_OK;
    }
    std::vector<uint4> hot(2 * n), cold(n);
    for (size_t o = 0; o < n; ++o) {
        std::memcpy(static_cast<void *>(&hot[2 * o]), &rec[o], 32);
        std::memcpy(static_cast<void *>(&cold[o]), reinterpret_cast<const char *>(&rec[o]) + 32, 16);
    }
    HIPCHK(hipMemcpyAsync(b.hot, hot.data(), sizeof(uint4) * hot.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(b.cold, cold.data(), sizeof(uint4) * cold.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // (the staging vectors end here)
    return DEM_OK;
}

static dem_status rec_download(dem_ctx *ctx, const RecBuf &b, std::vector<OwnerRec> &rec, hipStream_t s)
{
    const int64_t n = (int64_t)rec.size();
    if (!b.cold) {
        HIPCHK(hipMemcpyAsync(rec.data(), b.hot, sizeof(OwnerRec) * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return DEM_OK;
    }
    std::vector<uint4> hot(2 * n), cold(n);
    HIPCHK(hipMemcpyAsync(hot.data(), b.hot, sizeof(uint4) * hot.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(cold.data(), b.cold, sizeof(uint4) * cold.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t o = 0; o < n; ++o) {
        std::memcpy(&rec[o], &hot[2 * o], 32);
        std::memcpy(reinterpret_cast<char *>(&rec[o]) + 32, &cold[o], 16);
    }
    return DEM_OK;
}

dem_status dem_set_state(dem_ctx *ctx, const double *X, const double *q, const float *v, const float *w,
                         int64_t step, dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_set_state before dem_bind";
        return DEM_ERR_STATE;
    }
    ARGCHK(X && q && v && w, "X, q, v, w are required");
    hipStream_t s = S(stream);
    std::vector<OwnerRec> rec(ctx->No);
    std::vector<double> qd(4 * ctx->No);
    for (int64_t o = 0; o < ctx->No; ++o) {
        OwnerRec r{};
        uint32_t iv[3];
        for (int k = 0; k < 3; ++k) {
            ARGCHK(std::isfinite(X[3 * o + k]), "non-finite position");
            encode_axis(X[3 * o + k], ctx->org.o[k], &iv[k], &r.off[k]);
        }
        r.vox = pack_vox(iv[0], iv[1], iv[2]);
        double qq[4] = {q[4 * o], q[4 * o + 1], q[4 * o + 2], q[4 * o + 3]};
        double nn = std::sqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
        ARGCHK(nn > 0.5 && nn < 2.0, "quaternions must be (close to) unit length");
        for (int k = 0; k < 3; ++k) r.v[k] = v[3 * o + k];
        if (ctx->tmpl[o] < 0) {
            double R[9];
            host_rot(qq, R);
            for (int k = 0; k < 3; ++k)
                r.w[k] = (float)((R[3 * k] * w[3 * o] + R[3 * k + 1] * w[3 * o + 1]) + R[3 * k + 2] * w[3 * o + 2]);
            qd[4 * o] = 1.0;
            qd[4 * o + 1] = qd[4 * o + 2] = qd[4 * o + 3] = 0.0;
        } else {
            for (int k = 0; k < 3; ++k) r.w[k] = w[3 * o + k];
            for (int k = 0; k < 4; ++k) qd[4 * o + k] = qq[k];
        }
        r.mass = ctx->mass[o];
        if (ctx->famfixed[ctx->ofam[o]]) {
            // owners of fixed families keep zero velocity
            for (int k = 0; k < 3; ++k) r.v[k] = r.w[k] = 0.0f;
        }
        rec[o] = r;
    }
    // the fused step does not rewrite the records of fixed owners: both
    // buffers start equal
    for (const RecBuf &b : {ctx->rec, ctx->rec_alt}) {
        const dem_status st = rec_upload(ctx, b, rec, s);
        if (st != DEM_OK) return st;
    }
    HIPCHK(hipMemcpyAsync(ctx->q, qd.data(), sizeof(double) * 4 * ctx->No, hipMemcpyHostToDevice, s));
    // the fused step leaves the orientations of single-sphere systems alone,
    // so both buffers hold them
    HIPCHK(hipMemcpyAsync(ctx->q_alt, qd.data(), sizeof(double) * 4 * ctx->No, hipMemcpyHostToDevice, s));
    DevCounters z{};
    HIPCHK(hipMemcpyAsync(ctx->ctr, &z, sizeof(DevCounters), hipMemcpyHostToDevice, s));
    clear_set(ctx, 0, s);
    clear_set(ctx, 1, s);
    ctx->step = step;
    rebuild_dormant_index(ctx, s);
    HIPCHK(hipStreamSynchronize(s));
    ctx->has_state = true;
    ctx->cur = 0;
    ctx->sched_init = false;
    ctx->prep_valid = false;
    ctx->pending = false;
    return DEM_OK;
}

dem_status dem_get_state(dem_ctx *ctx, double *X, double *q, float *v, float *w, int64_t *step,
                         dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_get_state before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    std::vector<double> qd(4 * ctx->No);
    std::vector<OwnerRec> rec(ctx->No);
    const dem_status st = rec_download(ctx, ctx->rec, rec, s);
    if (st != DEM_OK) return st;
    HIPCHK(hipMemcpyAsync(qd.data(), ctx->q, sizeof(double) * 4 * ctx->No, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t o = 0; o < ctx->No; ++o) {
        const OwnerRec &r = rec[o];
        for (int k = 0; k < 3; ++k) {
            if (X) X[3 * o + k] = decode_axis(r.vox, r.off[k], ctx->org.o[k], k);
            if (v) v[3 * o + k] = r.v[k];
            if (w) w[3 * o + k] = r.w[k];
        }
        if (q)
            for (int k = 0; k < 4; ++k) q[4 * o + k] = qd[4 * o + k];
    }
    if (step) *step = ctx->step;
    return DEM_OK;
}

dem_status dem_bin(dem_ctx *ctx, dem_stream stream, uint32_t *sorted_keys, uint32_t *sorted_ids)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_bin before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    DetectArgs a = detect_args(ctx, ctx->P.margin, ctx->step);
    a.famdormant = nullptr;   // every sphere binned
    launch_bin(a, ctx->cdD, s);
    HIPCHK(hipGetLastError());
    if (sorted_keys || sorted_ids) {
        if (sorted_keys)
            HIPCHK(hipMemcpyAsync(sorted_keys, ctx->cdD.keys, 4 * ctx->Ns, hipMemcpyDeviceToHost, s));
        if (sorted_ids)
            HIPCHK(hipMemcpyAsync(sorted_ids, ctx->cdD.vals, 4 * ctx->Ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return DEM_OK;
}

static void flush_remap(dem_ctx *ctx, hipStream_t s);

static dem_status detect_now(dem_ctx *ctx, double margin, hipStream_t s, int target)
{
    // the buffer written here may be the one a deferred adoption still
    // carries its history from
    flush_remap(ctx, s);
    DetectArgs a = detect_args(ctx, margin, ctx->step);
    auto *tp = stage_begin(ctx, 2, s);
    launch_detect(a, ctx->cdD, ctx->acs[target], ctx->cap, ctx->ctr, target, s);
    stage_end(tp, s);
    HIPCHK(hipGetLastError());
    return DEM_OK;
}

// Carries the history of a deferred adoption over now (k_remap).
static void flush_remap(dem_ctx *ctx, hipStream_t s)
{
    if (ctx->rm_from < 0) return;
    auto *tp = stage_begin(ctx, 3, s);
    launch_remap(ctx->acs[ctx->rm_from], ctx->acs[ctx->cur], ctx->Ns, ctx->ctr, ctx->cur, ctx->rolling ? 1 : 0, s);
    stage_end(tp, s);
    ctx->rm_from = -1;
}

// Makes buffer `target` the set in use, its history carried over from the
// set in use before.  With `defer` (dem_step, right before a fused step)
// the carrying over is left to that step, which looks each touching pair's
// history up in the previous set: one launch and its stream transitions
// fewer per adoption.
static dem_status adopt(dem_ctx *ctx, int target, hipStream_t s, bool defer = false)
{
    flush_remap(ctx, s);
    if (defer && ctx->P.dyn_path != 1) {
        ctx->rm_from = ctx->cur;
    } else {
        auto *tp = stage_begin(ctx, 3, s);
        launch_remap(ctx->acs[ctx->cur], ctx->acs[target], ctx->Ns, ctx->ctr, target, ctx->rolling ? 1 : 0, s);
        stage_end(tp, s);
    }
    HIPCHK(hipGetLastError());
    ctx->cur = target;
    ++ctx->adopt_epoch;
    return DEM_OK;
}

dem_status dem_detect_contacts(dem_ctx *ctx, double margin, dem_stream stream, int64_t *n_contacts)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_detect_contacts before dem_bind";
        return DEM_ERR_STATE;
    }
    ARGCHK(margin >= 0.0 && margin <= ctx->P.margin * (1.0 + 1e-12), "margin must be in [0, params.margin]");
    hipStream_t s = S(stream);
    int target = 1 - ctx->cur;
    dem_status st = detect_now(ctx, margin, s, target);
    if (st != DEM_OK) return st;
    st = adopt(ctx, target, s);
    if (st != DEM_OK) return st;
    ctx->sched_init = false;
    ctx->prep_valid = false;
    ctx->pending = false;
    if (n_contacts) {
        st = read_counters(ctx, s);
        if (st != DEM_OK) return st;
        if (ctx->h_ctr->overflow[target]) {
            *n_contacts = ctx->h_ctr->required;
            ctx->err = "contact capacity exceeded";
            return DEM_ERR_CAPACITY;
        }
        *n_contacts = ctx->h_ctr->n_contacts[target];
    }
    return DEM_OK;
}

// The static index of the dormant spheres from the current state (their
// records do not change while the tags stay).
static void rebuild_dormant_index(dem_ctx *ctx, hipStream_t s)
{
    if (!ctx->has_dormant) return;
    DetectArgs a = detect_args(ctx, ctx->P.margin, ctx->step);
    launch_dormant_index(a, ctx->cdD, ctx->d_dcell_start, ctx->d_dcand, ctx->d_dcandf, s);
}

dem_status dem_set_families(dem_ctx *ctx, const dem_families *fam, dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_set_families before dem_bind";
        return DEM_ERR_STATE;
    }
    std::vector<uint8_t> off(65536, 0), fx(256, 0), of(ctx->No, 0), mf(ctx->NM, 0);
    if (fam && fam->pair_off) {
        for (int a = 0; a < 256; ++a)
            for (int b = 0; b < 256; ++b) {
                const uint8_t v = fam->pair_off[256 * a + b];
                ARGCHK(v <= 1, "pair_off entries must be 0 or 1");
                ARGCHK(v == fam->pair_off[256 * b + a], "pair_off must be symmetric");
                off[256 * a + b] = v;
            }
    }
    if (fam && fam->fixed)
        for (int a = 0; a < 256; ++a) fx[a] = fam->fixed[a] ? 1 : 0;
    if (fam && fam->owner_family) std::copy(fam->owner_family, fam->owner_family + ctx->No, of.begin());
    if (fam && fam->mesh_family) std::copy(fam->mesh_family, fam->mesh_family + ctx->NM, mf.begin());
    for (int w = 0; w < ctx->W; ++w) ctx->walls[w].family = (fam && fam->wall_family) ? fam->wall_family[w] : 0;
    ctx->pairoff.swap(off);
    ctx->famfixed.swap(fx);
    ctx->ofam.swap(of);
    ctx->mesh_family.swap(mf);
    ctx->has_pairoff = std::any_of(ctx->pairoff.begin(), ctx->pairoff.end(), [](uint8_t v) { return v != 0; });
    ctx->has_fixed = false;
    std::vector<uint8_t> used(256, 0);
    for (int64_t o = 0; o < ctx->No; ++o) {
        ctx->has_fixed = ctx->has_fixed || ctx->famfixed[ctx->ofam[o]];
        used[ctx->ofam[o]] = 1;
    }
    // dormant families: fixed, and switched off with every fixed family in
    // use and with every wall and mesh family -- their spheres can only touch
    // owners of the other families, which find them in the dormant index
    std::vector<uint8_t> other(256, 0);
    for (int w = 0; w < ctx->W; ++w) other[ctx->walls[w].family] = 1;
    for (uint8_t f : ctx->mesh_family) other[f] = 1;
    ctx->famdormant.assign(256, 0);
    ctx->has_dormant = false;
    for (int f = 0; f < 256; ++f) {
        if (!ctx->famfixed[f]) continue;
        bool d = true;
        for (int g = 0; g < 256 && d; ++g) {
            if ((used[g] && ctx->famfixed[g]) || other[g]) d = ctx->pairoff[256 * f + g] != 0;
        }
        ctx->famdormant[f] = d ? 1 : 0;
        ctx->has_dormant = ctx->has_dormant || (d && used[f]);
    }
    hipStream_t s = S(stream);
    HIPCHK(hipMemcpyAsync(ctx->d_ofam, ctx->ofam.data(), ctx->No, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_pairoff, ctx->pairoff.data(), 65536, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_famfixed, ctx->famfixed.data(), 256, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_famdormant, ctx->famdormant.data(), 256, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_walls, ctx->walls.data(), sizeof(WallDev) * ctx->walls.size(), hipMemcpyHostToDevice,
                          s));
    if (!ctx->has_state) {
        HIPCHK(hipStreamSynchronize(s));
        return DEM_OK;
    }
    if (ctx->has_fixed)
        launch_fix_owners(ctx->rec, ctx->rec_alt, ctx->q, ctx->q_alt, ctx->d_ofam, ctx->d_famfixed, ctx->No, s);
    rebuild_dormant_index(ctx, s);
    // the set in use was built under the old tags: rebuild it from the
    // current state (history of the pairs still listed carried over)
    int64_t n = 0;
    dem_status st = dem_detect_contacts(ctx, ctx->P.margin, stream, &n);
    if (st != DEM_OK) return st;
    HIPCHK(hipStreamSynchronize(s));
    return DEM_OK;
}

dem_status dem_forces(dem_ctx *ctx, dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_forces before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    DynArgs a = dyn_args(ctx, ctx->step);
    a.poses = dyn_poses(ctx, ctx->step, s);
    launch_force(a, ctx->acs[ctx->cur], ctx->sb, ctx->ctr, s);
    launch_fold_integrate(a, ctx->acs[ctx->cur], ctx->sb, ctx->ctr, 0, s);
    HIPCHK(hipGetLastError());
    return DEM_OK;
}

dem_status dem_get_forces(dem_ctx *ctx, float *F_owner, float *T_owner, float *F_contact, int64_t cap,
                          dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_get_forces before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    dem_status st = read_counters(ctx, s);
    if (st != DEM_OK) return st;
    int64_t No = ctx->No;
    std::vector<float> tmp(3 * No);
    if (F_owner) {
        HIPCHK(hipMemcpy(tmp.data(), ctx->sb.Fo, 12 * No, hipMemcpyDeviceToHost));
        for (int64_t o = 0; o < No; ++o)
            for (int k = 0; k < 3; ++k) F_owner[3 * o + k] = tmp[k * No + o];
    }
    if (T_owner) {
        HIPCHK(hipMemcpy(tmp.data(), ctx->sb.To, 12 * No, hipMemcpyDeviceToHost));
        for (int64_t o = 0; o < No; ++o)
            for (int k = 0; k < 3; ++k) T_owner[3 * o + k] = tmp[k * No + o];
    }
    if (F_contact) {
        int64_t n = ctx->h_ctr->n_contacts[ctx->cur];
        ARGCHK(cap >= n, "F_contact capacity smaller than the contact count");
        std::vector<float> b(3 * (size_t)std::max<int64_t>(n, 1));
        for (int k = 0; k < 3; ++k)
            if (n) HIPCHK(hipMemcpy(b.data() + k * n, ctx->sb.bF + k * ctx->cap, 4 * n, hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < n; ++c)
            for (int k = 0; k < 3; ++k) F_contact[3 * c + k] = -b[k * n + c];
    }
    return DEM_OK;
}

dem_status dem_get_contacts(dem_ctx *ctx, uint64_t *keys, float *hist, int64_t cap, int64_t *n,
                            dem_stream stream)
{
    if (!ctx || !n) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_get_contacts before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    const AcsBuf &a = ctx->acs[ctx->cur];
    std::vector<uint32_t> start(ctx->Ns + 1);
    HIPCHK(hipMemcpyAsync(start.data(), a.start, 4 * (ctx->Ns + 1), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t total = start[ctx->Ns];
    *n = total;
    if (total > ctx->cap) {
        ctx->err = "active set overflowed its capacity";
        return DEM_ERR_CAPACITY;
    }
    if (cap < total) {
        ctx->err = "output capacity smaller than the contact count";
        return DEM_ERR_CAPACITY;
    }
    std::vector<uint32_t> j(std::max<int64_t>(total, 1));
    std::vector<float> h(4 * (size_t)std::max<int64_t>(total, 1), 0.0f);
    if (total) {
        HIPCHK(hipMemcpyAsync(j.data(), a.j, 4 * total, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h.data(), a.hx, 4 * total, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h.data() + total, a.hy, 4 * total, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(h.data() + 2 * total, a.hz, 4 * total, hipMemcpyDeviceToHost, s));
        if (ctx->rolling) HIPCHK(hipMemcpyAsync(h.data() + 3 * total, a.hw, 4 * total, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    for (int64_t i = 0; i < ctx->Ns; ++i)
        for (uint32_t c = start[i]; c < start[i + 1]; ++c) {
            if (keys) keys[c] = ((uint64_t)i << 32) | (uint64_t)j[c];
            if (hist)
                for (int k = 0; k < 4; ++k) hist[4 * (size_t)c + k] = h[k * total + c];
        }
    return DEM_OK;
}

dem_status dem_set_contacts(dem_ctx *ctx, const uint64_t *keys, const float *hist, int64_t n,
                            dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_set_contacts before dem_bind";
        return DEM_ERR_STATE;
    }
    ARGCHK(n >= 0 && (n == 0 || keys), "keys required");
    if (n > ctx->cap) {
        ctx->err = "more contacts than the bound capacity";
        return DEM_ERR_CAPACITY;
    }
    hipStream_t s = S(stream);
    std::vector<uint32_t> start(ctx->Ns + 1, 0), j(std::max<int64_t>(n, 1));
    std::vector<float> h(4 * (size_t)std::max<int64_t>(n, 1), 0.0f);
    for (int64_t c = 0; c < n; ++c) {
        uint64_t key = keys[c];
        int64_t i = (int64_t)(key >> 32), jj = (int64_t)(key & 0xffffffffu);
        ARGCHK(c == 0 || keys[c - 1] < key, "keys must be strictly ascending");
        ARGCHK(i < ctx->Ns, "key sphere id out of range");
        ARGCHK((jj > i && jj < ctx->Ns) || (jj >= ctx->Ns && jj < ctx->Ns + ctx->W + ctx->NF),
               "key partner out of range");
        start[i + 1]++;
        j[c] = (uint32_t)jj;
        if (hist)
            for (int k = 0; k < 4; ++k) h[k * n + c] = hist[4 * c + k];
    }
    for (int64_t i = 0; i < ctx->Ns; ++i) start[i + 1] += start[i];
    int b = ctx->cur;
    AcsBuf &a = ctx->acs[b];
    HIPCHK(hipMemcpyAsync(a.start, start.data(), 4 * (ctx->Ns + 1), hipMemcpyHostToDevice, s));
    if (n) {
        HIPCHK(hipMemcpyAsync(a.j, j.data(), 4 * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(a.hx, h.data(), 4 * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(a.hy, h.data() + n, 4 * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(a.hz, h.data() + 2 * n, 4 * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(a.hw, h.data() + 3 * n, 4 * n, hipMemcpyHostToDevice, s));
    }
    launch_blists(a, ctx->Ns, ctx->cap, ctx->cdD.partials, s);
    launch_owner_flags(a, ctx->has_clumps ? ctx->d_sph0 : nullptr, ctx->No, ctx->Ns, ctx->cap, ctx->d_ofam,
                       ctx->has_fixed ? ctx->d_famfixed : nullptr, s, owner_list_wanted(ctx), ctx->cdD.partials);
    HIPCHK(hipGetLastError());
    uint32_t nn = (uint32_t)n, zero = 0;
    HIPCHK(hipMemcpyAsync(&ctx->ctr->n_contacts[b], &nn, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(&ctx->ctr->overflow[b], &zero, 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    ctx->sched_init = false;
    ctx->prep_valid = false;
    ctx->pending = false;
    return DEM_OK;
}

dem_status dem_count_missing(dem_ctx *ctx, dem_stream stream, int64_t *missing)
{
    if (!ctx || !missing) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_count_missing before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    launch_fill_u32(&ctx->ctr->miss, 1, 0u, s);
    DetectArgs a = detect_args(ctx, 0.0, ctx->step);
    launch_judge(a, ctx->cdD, ctx->acs[ctx->cur], ctx->cap, ctx->ctr, s);
    HIPCHK(hipGetLastError());
    dem_status st = read_counters(ctx, s);
    if (st != DEM_OK) return st;
    *missing = ctx->h_ctr->miss;
    return DEM_OK;
}

// ---------------------------------------------------------------------------
// the step loop
// ---------------------------------------------------------------------------
int64_t learned_interval(dem_ctx *ctx, hipStream_t s);
static void prepare_decision(dem_ctx *ctx, hipStream_t s);

// Adaptive schedule: the latency of the next cycle from the timing of a
// finished one.  The detection of cycle c took d_cd from its work order; the
// dynamics stream took d_dyn to reach the adoption step (before waiting).
// The smallest latency at which the dynamics would not have waited is
// lam_c d_cd / d_dyn; 10 % is added.  A cycle whose margin hit its cap
// shrinks the latency instead (a shorter n_max needs a smaller margin).
static void adapt_latency(dem_ctx *ctx)
{
    const int last = ctx->cyc_pos;                 // most recent work order
    const int prev = (last + 3) % 4, prev2 = (last + 2) % 4;
    // bound how far the host runs ahead: the cycle two work orders back
    // has been adopted on the device
    if (ctx->cyc[prev2].adopted) hipEventSynchronize(ctx->cyc[prev2].adopt);
    int use = -1;
    if (ctx->cyc[prev].adopted && hipEventQuery(ctx->cyc[prev].adopt) == hipSuccess) use = prev;
    else if (ctx->cyc[prev2].adopted) use = prev2;
    if (use < 0) return;
    dem_ctx::Cycle &c = ctx->cyc[use];
    if (hipEventQuery(c.cd) != hipSuccess) return;
    float d_cd = 0.f, d_dyn = 0.f;
    if (hipEventElapsedTime(&d_cd, c.wo, c.cd) != hipSuccess) return;
    if (hipEventElapsedTime(&d_dyn, c.wo, c.adopt) != hipSuccess || !(d_dyn > 0.f)) return;
    int lam;
    if (ctx->h_capped[use]) {
        lam = c.lam - 1;
    } else {
        lam = (int)std::ceil((double)c.lam * (double)d_cd / (double)d_dyn * 1.1);
    }
    const int lmax = std::max(1, ctx->P.cd_interval_max);
    ctx->lam_cur = std::min(std::max(lam, 1), lmax);
}

// Issues a work order at step n: the detection front on the dynamics stream
// (it reads the state of step n), the rest on the detection stream.
// Returns the latency (steps to adoption) of this cycle.
static int64_t issue_work_order(dem_ctx *ctx, hipStream_t dyn, hipStream_t kin, int64_t n)
{
    const dem_params &P = ctx->P;
    // the previous order's detection-stream part is enqueued (its workspace
    // and events are reused here)
    kin_join(ctx);
    // the order's buffer may be the one a deferred adoption still carries
    // its history from (an order at the adoption step)
    flush_remap(ctx, dyn);
    // (the learned interval's feature pass, which decided this order, has
    // written the snapshot its next features are measured against)
    int64_t lam = P.cd_latency;
    int target = 1 - ctx->cur;
    DetectArgs a = detect_args(ctx, P.margin, n);
    dem_ctx::Cycle *cy = nullptr;
    if (P.cd_mode == DEM_CD_ADAPTIVE) {
        adapt_latency(ctx);
        lam = ctx->lam_cur;
        const double g = std::sqrt(P.gravity[0] * P.gravity[0] + P.gravity[1] * P.gravity[1] +
                                   P.gravity[2] * P.gravity[2]);
        launch_reduce_max(dyn_args(ctx, n), ctx->ctr, dyn);
        launch_adaptive_margin(ctx->ctr, 2.0 * (double)lam * P.dt, g, P.margin, std::max(ctx->vmesh, ctx->vwall),
                               dyn);
        const int slot = (ctx->cyc_pos + 1) % 4;
        hipMemcpyAsync(&ctx->h_capped[slot], &ctx->ctr->capped, sizeof(uint32_t), hipMemcpyDeviceToHost, dyn);
        cy = &ctx->cyc[slot];
        hipEventRecord(cy->wo, dyn);
        cy->lam = (int)lam;
        cy->issued = true;
        cy->adopted = false;
        ctx->cyc_pos = slot;
        a.margin_dev = &ctx->ctr->margin;
    }
    // the work order: the first binning kernel reads the state of step n on
    // the dynamics stream (centres, bin keys and candidate records are the
    // snapshot); the rest of the detection runs on the detection stream
    if (!ctx->cdk_zeroed) {
        launch_zero3(ctx->cdK.cell_count, (int64_t)ctx->grid.nbins + 1, nullptr, 0, nullptr, 0, dyn);
        ctx->cdk_zeroed = true;
    }
    // in single-sphere runs without fixed families (one-pass bin sort, fused
    // dynamics) the binning step rides on the step of this iteration, which
    // reads the same state: one launch and one pass over the state fewer
    // (not with the timing-adaptive latency: it times each order from its
    // event to the end of its detection, and a binning step inside a whole
    // dynamics step skews that measure; measured on the mixer, the latency
    // then settles at half its value and the orders double)
    // Only when the adoption comes at a later step: with lambda = 0 the set
    // is adopted before this step's kernel runs, so its binning must be done
    // (and the detection chain enqueued) before that.
    const bool fuse = !ctx->has_clumps && !ctx->has_fixed && ctx->cdK.sort_mode == 0 && P.dyn_path != 1 &&
                      ctx->rm_from < 0 && P.cd_mode != DEM_CD_ADAPTIVE && lam > 0;
    if (!fuse) {
        auto *tf = stage_begin(ctx, 2, dyn);
        launch_detect_front(a, ctx->cdK, ctx->acs[target], dyn);
        if (tf) {
            stage_end(tf, dyn);
            tf->count = 0;   // one detection is counted once, with its back part
        }
    }
    auto *tp = stage_slot(ctx, 2);
    auto back = [ctx, a, target, kin, tp, cy]() {
        hipStreamWaitEvent(kin, ctx->ev_wo, 0);
        if (tp) hipEventRecord(tp->a, kin);
        launch_detect_back(a, ctx->cdK, ctx->acs[target], ctx->cap, ctx->ctr, target, kin);
        if (tp) hipEventRecord(tp->b, kin);
        if (cy) hipEventRecord(cy->cd, kin);
        hipEventRecord(ctx->ev_cd, kin);
    };
    // on a separate detection stream the launches go out from the other
    // host thread; on one stream they must keep their place in its order
    auto finish = [ctx, dyn, kin, back]() {
        hipEventRecord(ctx->ev_wo, dyn);
        if (kin != dyn)
            kin_post(ctx, back);
        else
            back();
    };
    if (fuse) {
        ctx->wo_fused = true;
        ctx->wo_finish = finish;
        ctx->wo_args = a;
        ctx->wo_target = target;
    } else {
        finish();
    }
    ctx->pending = true;
    ctx->pend_buf = target;
    ctx->pend_swap = n + lam;
    if (ctx->n_wo > 0) ctx->interval_sum += (double)(n - ctx->last_wo);
    ctx->last_wo = n;
    ctx->n_wo++;
    return lam;
}

// A work order left waiting for its step (dem_step returned before it):
// its binning step runs as a kernel of its own, then the rest goes out.
static void flush_work_order(dem_ctx *ctx, hipStream_t dyn)
{
    if (!ctx->wo_fused) return;
    launch_detect_front(ctx->wo_args, ctx->cdK, ctx->acs[ctx->wo_target], dyn);
    ctx->wo_fused = false;
    ctx->wo_finish();
    ctx->wo_finish = nullptr;
}

// When dem_step returns, by any path: a pending work order and a deferred
// carrying over of history are done, and the detection-stream thread
// joined.
struct StepGuard {
    dem_ctx *ctx;
    hipStream_t dyn;
    ~StepGuard()
    {
        flush_work_order(ctx, dyn);
        flush_remap(ctx, dyn);
        kin_join(ctx);
    }
};

dem_status dem_step(dem_ctx *ctx, int64_t n_steps, dem_stream dyn_, dem_stream kin_, dem_step_stats *stats)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_step before dem_bind";
        return DEM_ERR_STATE;
    }
    ARGCHK(n_steps >= 0, "n_steps must be >= 0");
    hipStream_t dyn = S(dyn_), kin = kin_ ? S(kin_) : dyn;
    StepGuard guard{ctx, dyn};
    auto t0 = std::chrono::steady_clock::now();
    const dem_params &P = ctx->P;
    int64_t cds = 0, swaps = 0, misses = 0, repairs = 0;
    const int64_t step0 = ctx->step;
    dem_status result = DEM_OK;
    if (ctx->run) {
        // a run left open by a call that returned early is discarded
        ctx->run->kind = -1;
        ctx->run = nullptr;
        ctx->run_len = 0;
    }
    ctx->run_due = false;
    drain_all(ctx);
    for (int k = 0; k < 5; ++k) {
        ctx->stage_ms[k] = 0.0;
        ctx->stage_n[k] = 0;
    }
    unsigned long long cs0 = 0;
    {
        dem_status st0 = read_counters(ctx, dyn);
        if (st0 != DEM_OK) return st0;
        cs0 = ctx->h_ctr->contact_steps;
    }
    if (ctx->n_wo == 0) ctx->interval_sum = 0.0;
    // the chain of pair-skipping steps: its set (by adoption count) and the
    // step that may continue it (every call starts a new one)
    uint64_t gap_epoch = 0;
    int64_t gap_next = -1;
    for (int64_t t = 0; t < n_steps; ++t) {
        const int64_t n = ctx->step;
        {
            // close a timed run before a step that enqueues other work on
            // the dynamics stream
            const bool busy = P.cd_mode == DEM_CD_EVERY || !ctx->sched_init || P.judge || n == ctx->next_wo ||
                              (P.cd_mode == DEM_CD_LEARNED && n + 1 == ctx->next_wo) ||
                              (ctx->pending && n == ctx->pend_swap);
            if (busy) run_close(ctx, dyn);
        }
        if (P.cd_mode == DEM_CD_EVERY) {
            int target = 1 - ctx->cur;
            dem_status st = detect_now(ctx, 0.0, dyn, target);
            if (st != DEM_OK) return st;
            st = adopt(ctx, target, dyn, true);
            if (st != DEM_OK) return st;
            ++cds;
            ++swaps;
        } else {
            if (!ctx->sched_init) {
                if (ctx->pending) {
                    kin_join(ctx);
                    hipStreamWaitEvent(dyn, ctx->ev_cd, 0);
                }
                int target = 1 - ctx->cur;
                dem_status st = detect_now(ctx, P.margin, dyn, target);
                if (st != DEM_OK) return st;
                st = adopt(ctx, target, dyn, true);
                if (st != DEM_OK) return st;
                ++cds;
                ++swaps;
                ctx->sched_init = true;
                ctx->pending = false;
                ctx->last_wo = n;
                ctx->n_wo = 1;
                ctx->interval_sum = 0.0;
                if (P.cd_mode == DEM_CD_LEARNED) {
                    snapshot_write(ctx->rec, ctx->fref, ctx->No, dyn);
                    ctx->snap_step = n;
                    ctx->prep_valid = false;
                }
                // the first interval is the fixed one: the learned interval's
                // features (and its analytic fallback's top speed) measure
                // motion since the previous work order, and there is none yet
                int64_t k = P.cd_mode == DEM_CD_ADAPTIVE ? 1 : std::min(P.cd_interval, P.cd_interval_max);
                ctx->next_wo = n + k;
                if (P.cd_mode == DEM_CD_ADAPTIVE) {
                    ctx->lam_cur = std::max(1, P.cd_latency);
                    for (auto &c : ctx->cyc) c.issued = c.adopted = false;
                }
            } else {
                int64_t k_next = -1;
                if (P.cd_latency == 0 && n == ctx->next_wo) {
                    k_next = P.cd_mode == DEM_CD_LEARNED ? learned_interval(ctx, dyn) : P.cd_interval;
                    issue_work_order(ctx, dyn, kin, n);
                    ++cds;
                }
                bool swap_due = ctx->pending && n == ctx->pend_swap;
                if (swap_due && P.cd_mode == DEM_CD_ADAPTIVE) {
                    dem_ctx::Cycle &c = ctx->cyc[ctx->cyc_pos];
                    hipEventRecord(c.adopt, dyn);
                    c.adopted = true;
                }
                if (swap_due) {
                    kin_join(ctx);
                    hipStreamWaitEvent(dyn, ctx->ev_cd, 0);
                }
                if (P.judge) {
                    int cand = swap_due ? ctx->pend_buf : ctx->cur;
                    launch_fill_u32(&ctx->ctr->miss, 1, 0u, dyn);
                    DetectArgs a = detect_args(ctx, 0.0, n);
                    launch_judge(a, ctx->cdD, ctx->acs[cand], ctx->cap, ctx->ctr, dyn);
                    dem_status st = read_counters(ctx, dyn);
                    if (st != DEM_OK) return st;
                    uint32_t miss = ctx->h_ctr->miss;
                    if (miss > 0) {
                        misses += miss;
                        ++repairs;
                        if (!P.repair) {
                            ctx->err = "judge found contacts missing from the active set";
                            result = DEM_ERR_MISSED;
                            break;
                        }
                        if (ctx->pending && !swap_due) {
                            kin_join(ctx);
                            hipStreamWaitEvent(dyn, ctx->ev_cd, 0);
                        }
                        int target = 1 - ctx->cur;
                        st = detect_now(ctx, P.margin, dyn, target);
                        if (st != DEM_OK) return st;
                        ++cds;
                        ctx->pending = false;
                        swap_due = true;
                        ctx->pend_buf = target;
                        int64_t k = P.cd_mode == DEM_CD_LEARNED
                                        ? learned_interval(ctx, dyn)
                                        : (P.cd_mode == DEM_CD_ADAPTIVE ? ctx->lam_cur : P.cd_interval);
                        ctx->next_wo = n + k;
                        k_next = -1;
                        ctx->last_wo = n;
                    }
                }
                if (swap_due) {
                    dem_status st = adopt(ctx, ctx->pend_buf, dyn, true);
                    if (st != DEM_OK) return st;
                    ctx->pending = false;
                    ++swaps;
                }
                if (P.cd_latency > 0 && n == ctx->next_wo && ctx->pending) {
                    // the previous detection is not adopted yet: its buffer
                    // and workspace are in use, so the order waits for the
                    // adoption step
                    ctx->next_wo = ctx->pend_swap;
                } else if (P.cd_latency > 0 && n == ctx->next_wo) {
                    int64_t k = P.cd_mode == DEM_CD_LEARNED ? learned_interval(ctx, dyn) : P.cd_interval;
                    if (P.cd_mode == DEM_CD_LEARNED && k < P.cd_latency) {
                        // the predicted horizon does not cover the latency of a
                        // delayed detection: detect now on the dynamics stream and
                        // use the set from this step on
                        const int target = 1 - ctx->cur;
                        dem_status st = detect_now(ctx, P.margin, dyn, target);
                        if (st != DEM_OK) return st;
                        st = adopt(ctx, target, dyn, true);
                        if (st != DEM_OK) return st;
                        if (ctx->n_wo > 0) ctx->interval_sum += (double)(n - ctx->last_wo);
                        ctx->last_wo = n;
                        ctx->n_wo++;
                        ++swaps;
                    } else {
                        const int64_t lam = issue_work_order(ctx, dyn, kin, n);
                        if (P.cd_mode == DEM_CD_ADAPTIVE) k = lam;   // the next order goes out at this adoption
                    }
                    ++cds;
                    ctx->next_wo = n + k;
                } else if (P.cd_latency == 0 && k_next > 0) {
                    ctx->next_wo = n + k_next;
                }
            }
        }
        // the learned schedule decides a work order due at the next step
        // from the state this step reads (enqueued before the step kernel)
        if (P.cd_mode == DEM_CD_LEARNED && ctx->sched_init && n + 1 == ctx->next_wo &&
            (!ctx->pending || ctx->pend_swap == n + 1))
            prepare_decision(ctx, dyn);
        DynArgs a = dyn_args(ctx, n);
        if (ctx->NM > 0) {
            // a refill of the pose ring is dynamics-stream work: no timed run spans it
            if (ctx->run && !(n >= ctx->pose_lo && n < ctx->pose_hi)) run_close(ctx, dyn);
            a.poses = dyn_poses(ctx, n, dyn);
        }
        // single kernels are bracketed by marker events, which wait for the
        // previous work on the stream; an empty kernel bracketed the same way
        // measures the markers' own overhead
        const bool split = P.dyn_path != 1 && step_is_split(a, ctx->acs[ctx->cur]);
        if (split) {
            // the two kernels of a split step are timed one event pair
            // each, every `timing`-th step, each pair followed by an empty
            // kernel bracketed the same way (the markers' own overhead)
            run_close(ctx, dyn);
            const bool gap = pair_skip_split_allowed(ctx, a);
            if (gap) a.gap = (gap_next == n && gap_epoch == ctx->adopt_epoch && !a.rm_start) ? 2 : 1;
            gap_next = gap ? n + 1 : -1;
            gap_epoch = ctx->adopt_epoch;
            SplitTiming tm{};
            dem_ctx::TimedPair *t1 = stage_slot(ctx, 1), *t0 = t1 ? stage_slot(ctx, 0) : nullptr;
            if (t1 && t0) tm = SplitTiming{t1->a, t1->b, t0->a, t0->b};
            launch_step_fused(a, ctx->rec_alt, ctx->q_alt, ctx->acs[ctx->cur], ctx->cap, ctx->ctr, dyn,
                              (t1 && t0) ? &tm : nullptr);
            if (t1 && t0) {
                if (auto *tn = stage_begin(ctx, 4, dyn)) {
                    launch_noop(dyn, nullptr, nullptr);
                    stage_end(tn, dyn);
                }
            } else {
                if (t1) t1->kind = -1;
                if (t0) t0->kind = -1;
            }
            ctx->rm_from = -1;
            std::swap(ctx->rec, ctx->rec_alt);
            std::swap(ctx->q, ctx->q_alt);
            swap_hist(ctx->acs[ctx->cur]);
        } else if (P.dyn_path != 1) {
            if (P.timing > 0 && n % P.timing == 0) ctx->run_due = true;
            if (!ctx->run && ctx->run_due) {
                bool open = P.cd_mode == DEM_CD_EVERY || P.judge;
                if (!open) {
                    int64_t next_busy = ctx->next_wo - (P.cd_mode == DEM_CD_LEARNED ? 1 : 0);
                    if (ctx->pending && ctx->pend_swap < next_busy) next_busy = ctx->pend_swap;
                    open = next_busy - n >= RUN_LAUNCHES;
                }
                if (open) {
                    ctx->run = stage_slot(ctx, 5);
                    if (ctx->run) hipEventRecord(ctx->run->a, dyn);
                    ctx->run_due = false;
                }
            }
            const bool gap = pair_skip_allowed(ctx, a);
            if (gap) a.gap = (gap_next == n && gap_epoch == ctx->adopt_epoch && !a.rm_start) ? 2 : 1;
            gap_next = gap ? n + 1 : -1;
            gap_epoch = ctx->adopt_epoch;
            if (!launch_step_fused(a, ctx->rec_alt, ctx->q_alt, ctx->acs[ctx->cur], ctx->cap, ctx->ctr, dyn)) {
                // (a work order's binning on the step right after an
                // adoption: issue_work_order never sets one up)
                ctx->err = "internal: no step kernel carries a work order's binning on this step";
                return DEM_ERR_STATE;
            }
            ctx->rm_from = -1;   // (the step carried the history over)
            if (ctx->wo_fused) {
                // (the step wrote the work order's binning)
                ctx->wo_fused = false;
                ctx->wo_finish();
                ctx->wo_finish = nullptr;
            }
            if (ctx->run && ++ctx->run_len == RUN_LAUNCHES) run_close(ctx, dyn);
            std::swap(ctx->rec, ctx->rec_alt);
            std::swap(ctx->q, ctx->q_alt);
            swap_hist(ctx->acs[ctx->cur]);
        } else {
            gap_next = -1;
            auto *tf = stage_begin(ctx, 0, dyn);
            launch_force(a, ctx->acs[ctx->cur], ctx->sb, ctx->ctr, dyn);
            stage_end(tf, dyn);
            auto *ti = stage_begin(ctx, 1, dyn);
            launch_fold_integrate(a, ctx->acs[ctx->cur], ctx->sb, ctx->ctr, 1, dyn);
            stage_end(ti, dyn);
        }
        if (P.dyn_path == 1) {
            if (auto *tn = stage_begin(ctx, 4, dyn)) {
                launch_noop(dyn, nullptr, nullptr);
                stage_end(tn, dyn);
            }
        }
        ctx->step = n + 1;
    }
    run_close(ctx, dyn);
    {
        DynArgs da = dyn_args(ctx, ctx->step);
        launch_reduce_max(da, ctx->ctr, dyn);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(kin_join(ctx));
    if (kin != dyn) HIPCHK(hipStreamSynchronize(kin));
    dem_status st = read_counters(ctx, dyn);
    if (st != DEM_OK) return st;
    const DevCounters &c = *ctx->h_ctr;
    if (c.stop_cd || c.div[0] || c.div[1]) {
        ctx->step = c.last_step_done > 0 ? c.last_step_done : step0;
        if (c.stop_cd) {
            ctx->err = "contact capacity exceeded during detection";
            result = DEM_ERR_CAPACITY;
        } else {
            ctx->err = "simulation diverged (NaN or speed above v_error_out)";
            result = DEM_ERR_DIVERGED;
        }
    }
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->steps = ctx->step - step0;
        stats->step = ctx->step;
        stats->cds = cds;
        stats->swaps = swaps;
        stats->misses = misses;
        stats->repairs = repairs;
        stats->n_contacts = c.n_contacts[ctx->cur];
        stats->required_capacity = c.required;
        float v2;
        uint32_t bits = c.maxv2[0];
        std::memcpy(&v2, &bits, 4);
        stats->max_speed = std::sqrt((double)v2);
        stats->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        stats->mean_interval = ctx->n_wo > 1 ? ctx->interval_sum / (double)(ctx->n_wo - 1)
                                             : (double)(P.cd_mode == DEM_CD_EVERY ? 1 : P.cd_interval);
        drain_all(ctx);
        for (int k = 0; k < 5; ++k) {
            stats->stage_ms[k] = ctx->stage_ms[k];
            stats->stage_n[k] = ctx->stage_n[k];
        }
        stats->mean_contacts = stats->steps > 0 ? (double)(c.contact_steps - cs0) / (double)stats->steps : 0.0;
    }
    return result;
}

void dem_destroy(dem_ctx *ctx)
{
    if (!ctx) return;
    kin_stop(ctx);
    if (ctx->h_ctr) hipHostFree(ctx->h_ctr);
    if (ctx->h_pred) hipHostFree(ctx->h_pred);
    if (ctx->ev_kdec) {
        hipEventSynchronize(ctx->ev_kdec);
        hipEventDestroy(ctx->ev_kdec);
    }
    if (ctx->h_kdec) hipHostFree(ctx->h_kdec);
    if (ctx->ev_wo) hipEventDestroy(ctx->ev_wo);
    if (ctx->ev_cd) hipEventDestroy(ctx->ev_cd);
    if (ctx->h_capped) hipHostFree(ctx->h_capped);
    for (auto &c : ctx->cyc) {
        if (c.wo) hipEventDestroy(c.wo);
        if (c.cd) hipEventDestroy(c.cd);
        if (c.adopt) hipEventDestroy(c.adopt);
    }
    for (auto &p : ctx->ring) {
        if (p.a) hipEventDestroy(p.a);
        if (p.b) hipEventDestroy(p.b);
    }
    // the staging may still feed a pending copy
    for (auto &e : ctx->ev_pose)
        if (e) hipEventSynchronize(e);
    if (ctx->h_pose_stage) hipHostFree(ctx->h_pose_stage);
    for (auto &e : ctx->ev_pose)
        if (e) hipEventDestroy(e);
    delete ctx;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned interval: features, MLP, policy, training-log tools
// ---------------------------------------------------------------------------
void mlp_forward(const float *params, const float *X, float *Y, int64_t n, hipStream_t s);
void launch_label_judge(const DetectArgs &a, CdWork &w, const uint32_t *lab_start, const uint32_t *lab_j,
                        int64_t cap, const uint32_t *cellmap, uint32_t *first_miss, uint32_t t, hipStream_t s);
void launch_detect_plain(const DetectArgs &a, CdWork &w, uint32_t *start, uint32_t *j, int64_t cap,
                         DevCounters *ctr, hipStream_t s);

static void run_features(dem_ctx *ctx, hipStream_t s, float *out, uint32_t *cell_ids)
{
    float tau = (float)(ctx->step - ctx->snap_step);
    float margin = (float)(ctx->P.margin > 0.0 ? ctx->P.margin : 1e-6);
    feature_pipeline(ctx->rec, ctx->fref, ctx->d_ovol, ctx->org, ctx->fgrid, (float)ctx->P.dt, margin, tau,
                     ctx->d_fraw, ctx->d_fflag, ctx->d_fpos, ctx->cdD.partials, ctx->d_cellmap, out, cell_ids, ctx->No,
                     s);
}

// Enqueues the learned schedule's decision from the current state on s
// (features against the snapshot, which the state then replaces; the
// network; the interval, with the analytic bound as its fallback), its
// copy to pinned host memory and an event after it.
static void enqueue_decision(dem_ctx *ctx, hipStream_t s, int ahead)
{
    const dem_params &P = ctx->P;
    LearnedArgs p;
    p.g = std::sqrt(P.gravity[0] * P.gravity[0] + P.gravity[1] * P.gravity[1] + P.gravity[2] * P.gravity[2]);
    p.margin = P.margin;
    p.dt = P.dt;
    p.safety = P.mlp_safety > 0.0 ? P.mlp_safety : 1.0;
    p.vgeom = std::max(ctx->vmesh, ctx->vwall);
    p.lam = P.cd_latency;
    p.kmax = P.cd_interval_max;
    p.use_model = ctx->mlp_set ? 1 : 0;
    p.moving = p.vgeom > 0.0 ? 1 : 0;
    p.speed_valid = ctx->step > 0 ? 1 : 0;
    p.ahead = ahead;
    const float tau = (float)(ctx->step - ctx->snap_step);
    const float margin = (float)(P.margin > 0.0 ? P.margin : 1e-6);
    const DynArgs da = dyn_args(ctx, ctx->step);
    learned_decide(ctx->rec, ctx->fref, ctx->d_ovol, ctx->org, ctx->fgrid, (float)P.dt, margin, tau, ctx->d_fraw,
                   ctx->d_mlp, ctx->d_pslot, ctx->d_blkmax, speed_slots(da), p, ctx->d_kdec, ctx->No, s);
    if (ctx->mlp_set) ctx->snap_step = ctx->step;
    hipMemcpyAsync(ctx->h_kdec, ctx->d_kdec, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    hipEventRecord(ctx->ev_kdec, s);
}

// The learned schedule one step ahead: the decision for a work order due at
// the next step is enqueued before this step's kernel, from the state this
// step reads, and read back at the order (the host waits only for a copy
// enqueued a whole step earlier, so the dynamics stream does not drain).
static void prepare_decision(dem_ctx *ctx, hipStream_t s)
{
    enqueue_decision(ctx, s, 1);
    ctx->prep_valid = true;
    ctx->prep_step = ctx->step;
}

// Decides the next detection interval at a work order (LEARNED mode): the
// MLP predicts, per cell, how many steps a set detected now stays complete;
// the minimum over cells, scaled by the model's calibrated safety factor,
// minus the adoption latency is the interval.  The analytic bound is the
// fallback when no model is installed or its prediction is not finite.
// Uses the decision prepared at the step before, if there is one; else
// enqueues it now and waits for it.
int64_t learned_interval(dem_ctx *ctx, hipStream_t s)
{
    if (!(ctx->prep_valid && ctx->prep_step + 1 == ctx->step)) enqueue_decision(ctx, s, 0);
    ctx->prep_valid = false;
    hipEventSynchronize(ctx->ev_kdec);
    const int64_t k = ctx->h_kdec[0];
    return k < 1 ? 1 : k;
}

extern "C" {

dem_status dem_mlp_set(dem_ctx *ctx, const float *params)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!params) {
        ctx->mlp_set = false;
        return DEM_OK;
    }
    ctx->mlp.assign(params, params + DEM_MLP_NPARAM);
    for (float f : ctx->mlp) ARGCHK(std::isfinite(f), "MLP parameters must be finite");
    ctx->mlp_set = true;
    if (ctx->bound) HIPCHK(hipMemcpy(ctx->d_mlp, params, sizeof(float) * DEM_MLP_NPARAM, hipMemcpyHostToDevice));
    return DEM_OK;
}

dem_status dem_snapshot(dem_ctx *ctx, dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_snapshot before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    snapshot_write(ctx->rec, ctx->fref, ctx->No, s);
    HIPCHK(hipGetLastError());
    ctx->snap_step = ctx->step;
    ctx->prep_valid = false;
    return DEM_OK;
}

dem_status dem_features(dem_ctx *ctx, float *out_dev, int64_t ncell_cap, int64_t *ncell, dem_stream stream)
{
    if (!ctx || !ncell) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_features before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    run_features(ctx, s, ctx->d_feat, ctx->d_fids);
    uint32_t nc = 0;
    HIPCHK(hipMemcpyAsync(&nc, ctx->d_fpos + ctx->fgrid.nbins, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *ncell = nc;
    if (out_dev) {
        if (ncell_cap < (int64_t)nc) {
            ctx->err = "feature output capacity too small";
            return DEM_ERR_CAPACITY;
        }
        if (nc) HIPCHK(hipMemcpyAsync(out_dev, ctx->d_feat, sizeof(float) * DEM_MLP_NFEAT * nc,
                                      hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return DEM_OK;
}

dem_status dem_feature_cells(dem_ctx *ctx, uint32_t *cell_ids, int64_t cap, uint32_t *owner_cell,
                             int64_t *n_cells_total, dem_stream stream)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_feature_cells before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    uint32_t nc = 0;
    HIPCHK(hipMemcpyAsync(&nc, ctx->d_fpos + ctx->fgrid.nbins, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (n_cells_total) *n_cells_total = (int64_t)ctx->fgrid.nbins;
    if (cell_ids) {
        ARGCHK(cap >= (int64_t)nc, "cell id capacity too small");
        if (nc) HIPCHK(hipMemcpy(cell_ids, ctx->d_fids, 4 * (size_t)nc, hipMemcpyDeviceToHost));
    }
    if (owner_cell) HIPCHK(hipMemcpy(owner_cell, ctx->d_cellmap, 4 * (size_t)ctx->No, hipMemcpyDeviceToHost));
    return DEM_OK;
}

dem_status dem_label_begin(dem_ctx *ctx, dem_stream stream, int64_t *n_contacts)
{
    if (!ctx) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_label_begin before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    DetectArgs a = detect_args(ctx, ctx->P.margin, ctx->step);
    launch_detect_plain(a, ctx->cdD, ctx->d_lab_start, ctx->d_lab_j, ctx->cap, ctx->ctr, s);
    HIPCHK(hipGetLastError());
    dem_status st = read_counters(ctx, s);
    if (st != DEM_OK) return st;
    if (n_contacts) *n_contacts = ctx->h_ctr->required;
    return DEM_OK;
}

dem_status dem_label_update(dem_ctx *ctx, uint32_t t, uint32_t *first_miss_dev, dem_stream stream)
{
    if (!ctx || !first_miss_dev) return DEM_ERR_ARG;
    if (!ctx->bound) {
        ctx->err = "dem_label_update before dem_bind";
        return DEM_ERR_STATE;
    }
    hipStream_t s = S(stream);
    DetectArgs a = detect_args(ctx, 0.0, ctx->step);
    launch_label_judge(a, ctx->cdD, ctx->d_lab_start, ctx->d_lab_j, ctx->cap, ctx->d_cellmap, first_miss_dev, t, s);
    HIPCHK(hipGetLastError());
    return DEM_OK;
}

dem_status dem_info(const dem_ctx *ctx, int64_t *vals, int64_t n)
{
    if (!ctx || !vals) return DEM_ERR_ARG;
    int64_t v[8] = {(int64_t)ctx->grid.nbins, (int64_t)ctx->fgrid.nbins, ctx->grid.nx, ctx->grid.ny,
                    ctx->grid.nz, ctx->sort_bits, ctx->cap, ctx->step};
    for (int64_t k = 0; k < n && k < 8; ++k) vals[k] = v[k];
    return DEM_OK;
}

}  // extern "C"
