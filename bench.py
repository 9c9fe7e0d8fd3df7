#!/usr/bin/env python3
"""Benchmark of the DEM hot path on one MI355X.

Workload (default): the large bed, about 60 M spheres in 32 M owners on a
7 mm lattice in a 2 x 2 m container -- 18 of every 32 owners single spheres
(r = 2 mm), the rest tri-sphere clumps (r = 2 mm, circumradius 4/3 mm) --
with an analytic cylinder (R = 0.1 m, L = 0.5 m) rolling across its top at
0.2 m/s; dt = 5e-6 s; margin 0.2 mm; delayed contact detection on a second
HIP stream at the learned interval (adoption latency 5 steps).  One "step"
is contact detection (amortised over its interval) + force + reduction +
integration for all spheres.  The same workload is also timed with the
fixed-margin schedule (every 10 steps), every-step detection, the learned
schedule's analytic fallback alone, and the paper's timing-adaptive policy.

Before any timing, every schedule runs once on a small system of the same
kind (clumps, walls, cylinder), so that each kernel the timed runs use has
been launched once in the process.

Prints one JSON line: sphere-steps/s of the learned schedule as `value`,
every schedule under `modes`, the roofline of the dominant kernel (live
HIP-event timing of that kernel over the timed region), the FP64 CPU oracle
timed on a bounded sample of the same workload, and the 1,000-sphere
every-step case run in full on the GPU and on the oracle side by side.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGES = ["k_force", "k_fold_integrate", "detect", "k_remap"]   # two-kernel dynamics
STAGES_FUSED = ["k_force", "k_step_fused", "detect", "k_remap"]  # fused dynamics (default)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1_000_000, help="spheres of the config-1 workload")
    ap.add_argument("--workload", default="config4",
                    help="config4 (headline: the 60 M-sphere bed) | config1 | config2 | config3: other sizes | "
                         "mixer: the bladed-mixer bed with a 2880-facet impeller | "
                         "activebox: the config-4 bed (quarter size) with an active box around the cylinder")
    ap.add_argument("--modes", default="learned,fixed,every,analytic,adaptive",
                    help="schedules: fixed (k steps), every (every step), learned (MLP interval), "
                         "analytic (the learned schedule's fallback bound alone, no network), "
                         "adaptive (work order at every adoption, latency adapted from timing, margin from n_max)")
    ap.add_argument("--no-judge", action="store_true", help="skip the judged (miss-counting) runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle steps of the CPU baseline (0: 50 for up to 2 M spheres, else 30)")
    ap.add_argument("--no-config0", action="store_true",
                    help="skip the 1,000-sphere every-step side-by-side run (GPU and oracle, 2,000 steps)")
    ap.add_argument("--no-prime", action="store_true", help="skip the small priming runs")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--lam", type=int, default=5)
    ap.add_argument("--no-pair-skip", action="store_true",
                    help="evaluate every pair of a dense single-sphere set every step (no skipping by gap keys)")
    ap.add_argument("--dyn-path", type=int, default=0,
                    help="dynamics: 0 one fused kernel per step, 1 force kernel + fold/integrate kernel, 2/3 fused with the history always/never staged in LDS")
    ap.add_argument("--timing", type=int, default=0,
                    help="time the dynamics kernel with HIP events every n-th step (0: steps // 4, at most 32)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    return ap.parse_args()


def algorithmic_bytes(stage, Ns, No, C, active, nbins, passes, clumps=True, rolling=False, n_clump=None, n_tri=0,
                      n_dormant=0, n_dormant_clump=0, n_dormant_sph=0, pair_keys=False):
    """Bytes one launch of a stage must move at minimum (unique data);
    `active` = spheres that appear in at least one contact:
    k_force: per sphere its row offset (4); per active sphere its record
      (16), its owner's record (48) and its A-side sums written (24); per
      contact the partner id (4), history read + write (24) and the B-side
      reaction written (24).
    k_step_fused: per owner its contact flag (1), the record read + write
      (96) and the inverse inertia (4 for single-sphere systems; else 16, and
      per clump owner the quaternion read + written 64); per active sphere
      its record, row and B-list offsets and its owner's sphere range (28);
      per contact the partner id (4), the new history written (12, 16 with
      contact age) and the B-list entry with its source sphere (8); the old
      history is read only for pairs that touch and is not counted (so the
      figure is a lower bound); with pair skipping (single spheres, dense
      sets) also each pair's gap key (4; it is rewritten only for the pairs
      the step evaluates, not counted);
      with meshes, each facet's vertices and mesh index (80).  An owner of a
      fixed family without contacts reads its flag only (1).
    k_fold_integrate: per owner the record read + write (96) and the inverse
      inertia: one isotropic value (4) when every owner is a single sphere,
      else three values and the template (16) plus the sphere range (4); per
      sphere the row and B-list offsets (8); per active sphere the A-side sums
      (24); per contact the B-list entry (4) and the reaction (24).
    detect: per sphere record + the owner record's hot part (48), key and
      slot in its bin (8) and candidate
      (32) written, radix passes (16 each), candidate gather (36 r + 16 w
      for the FP32 copy, + 32 w for the FP64 record in bin order with
      meshes),
      one traversal reading 32 B of candidates per neighbour-row hit, row
      count and offsets (8), staging (4 per partner), B lists (16); per
      contact partner id (4) and B-list bytes (16); the bin table (12 per bin);
      with meshes, per facet its vertices read (80), its world vertices, box
      and bin range written (144) and its row count and offset (8).  Only
      the spheres the detection bins count: the spheres of dormant owners
      are left out of it (the binned spheres' walks over the dormant index
      read data the caches serve and are not counted).
    k_remap: per sphere both row offsets (16); per contact new id (4), old id
      (4), history read (12) and written (12)."""
    if stage == "k_force":
        return Ns * 4 + active * 88 + C * 52
    if stage == "k_step_fused":
        nc = (No if n_clump is None else n_clump) if clumps else 0
        nc -= n_dormant_clump if clumps else 0
        return ((No - n_dormant) * (113 if clumps else 101) + n_dormant + nc * 64 + active * 28
                + C * ((28 if rolling else 24) + (4 if pair_keys else 0)) + n_tri * 80)
    if stage == "k_fold_integrate":
        return No * (116 if clumps else 100) + Ns * 8 + active * 24 + C * 28
    if stage == "detect":
        gather = 36 + 16 + (32 if n_tri > 0 else 0)
        return (Ns - n_dormant_sph) * (48 + 8 + 32 + 16 * passes + gather + 32 + 8 + 16) + C * 24 + nbins * 12 + n_tri * 232
    if stage == "k_remap":
        return Ns * 16 + C * 32
    raise ValueError(stage)


def stream_bytes(No, n_turn, n_spin=None):
    """k_step_free: per owner its contact flag (1) and the hot part of its
    record (position, velocity) read + written (64); per turning owner
    (nonzero angular velocity) the cold part of its record (angular
    velocity, mass) read + written (32) and its inertia and template (16),
    and per turning clump its orientation read + written (64): an owner at
    rest in rotation keeps its angular velocity and orientation in both
    buffers and needs none of them (without n_spin every owner is counted
    as turning).  Owners with contacts are counted here (their hot parts are
    read and written, then written again by k_step_listed)."""
    return No * 65 + (No if n_spin is None else n_spin) * 48 + n_turn * 64


def n_clump_share(sysm, rr):
    """Clumps among the owners with contacts, in proportion to their share
    of all owners (the split step's second kernel reads their orientation)."""
    No = sysm.n_owners
    frac = float(np.sum(np.asarray(sysm.own_tmpl) >= 0)) / max(No, 1)
    return int(round(rr["active_owners"] * frac))


def listed_bytes(n_own, n_clump, active, C, rolling):
    """k_step_listed: per owner with contacts its list entry (32: the owner,
    its first sphere and its spheres' row and B-list bounds), inertia and
    template (16) and record read + written (96); per clump among them its
    orientation read + written (64); per active sphere its record (20); per
    contact the partner id (4), the new history written (12, 16 with
    contact age) and the B-list entry with its source sphere (8)."""
    return n_own * 144 + n_clump * 64 + active * 20 + C * (28 if rolling else 24)


def kernel_sha(path, kernel):
    """Hash of one kernel's source text (its __global__ definition up to the
    closing brace in column 0), so counters taken on it stay valid while the
    kernel is unchanged."""
    lines = open(path).read().splitlines()
    start = next(i for i, l in enumerate(lines) if "__global__" in l and f" {kernel}(" in l)
    end = next(i for i in range(start, len(lines)) if lines[i].startswith("}"))
    return hashlib.sha256("\n".join(lines[start:end + 1]).encode()).hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 PMC summaries of this
    workload, if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        ent = d.get(kernel)
        if not ent:
            return None
        src = os.path.join(ROOT, "paper_2311_04648_amd", "csrc", ent["source"])
        if kernel_sha(src, kernel) != ent["kernel_sha"]:
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def make_ctx(dem, sysm, mode, args, mlp, judge, dyn_path=None):
    lib_mode = "learned" if mode == "analytic" else mode
    ctx = dem.DemContext(sysm, mode=lib_mode, k=args.k, lam=args.lam, judge=judge,
                         timing=0 if judge else args.timing, capacity=max(64, 8 * sysm.n_spheres), k_max=1024,
                         mlp_safety=args.mlp_safety, dyn_path=args.dyn_path if dyn_path is None else dyn_path,
                         pair_skip=not args.no_pair_skip)
    if mode == "learned":
        ctx.mlp_set(mlp)
    return ctx


def run_mode(dem, torch, sysm, mode, args, mlp=None, judge=False, turning=False):
    ctx = make_ctx(dem, sysm, mode, args, mlp, judge)
    ctx.set_state()
    dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
    if args.warmup:
        ctx.step(args.warmup, dyn=dyn, kin=kin)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = ctx.step(args.steps, dyn=dyn, kin=kin)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = ctx.info()
    keys, _ = ctx.get_contacts()
    ii = (keys >> np.uint64(32)).astype(np.int64)
    jj = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    active = np.unique(np.concatenate([ii, jj[jj < sysm.n_spheres]])).size
    act_own = np.unique(np.asarray(sysm.sph_owner)[np.unique(np.concatenate([ii, jj[jj < sysm.n_spheres]]))]).size
    n_turn = n_spin = None
    if turning:
        # owners turning at the end of the run: the streaming step reads the
        # inertia of these only, and the orientation of the clumps among them
        g = ctx.get_state()
        spin = np.any(np.asarray(g["W"]) != 0, axis=1)
        n_spin = int(np.sum(spin))
        n_turn = int(np.sum((np.asarray(sysm.own_tmpl) >= 0) & spin))
    ctx.close()
    del ctx
    return dict(seconds=t1 - t0, stats=stats, info=info, active=int(active), active_owners=int(act_own),
                n_turn=n_turn, n_spin=n_spin)


def priming_system(W, sysm):
    """A small system of the same kind as the workload (clumps or single
    spheres, walls, a cylinder, meshes, family tags), for one throwaway run
    of each schedule before any timing."""
    has_clumps = sysm.n_spheres != sysm.n_owners
    has_cyl = bool(np.any(np.asarray(sysm.wall_type) == 1))
    if sysm.n_tri:
        return W.small_mixer_bed(3, n=300)
    if has_clumps:
        small = W.small_clumps(2, n=400, with_cylinder=has_cyl, spacing=0.0085)
    else:
        small = W.small_spheres(2, n=512, vel=0.3)
    if np.asarray(getattr(sysm, "fam_fixed", np.zeros(0))).size:
        X = small.X
        lo = X.min(0) + 0.3 * (X.max(0) - X.min(0))
        small = W.active_box(small, lo, X.max(0) + 1.0)
    return small


def prime(dem, torch, W, sysm, modes, args, mlp):
    """Runs each schedule once on a small system of the workload's kind,
    long enough for work orders, adoptions and (learned) decisions, in each
    dynamics form the timed runs may pick."""
    small = priming_system(W, sysm)
    paths = [args.dyn_path]
    if args.dyn_path == 0:
        paths = [0, 3, 4] if small.n_spheres != small.n_owners else [0, 2, 3]
    dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
    for mode in modes:
        for path in paths:
            ctx = make_ctx(dem, small, mode, args, mlp, False, dyn_path=path)
            ctx.set_state()
            ctx.step(3 * (args.k + args.lam) + 4, dyn=dyn, kin=kin)
            ctx.close()
    torch.cuda.synchronize()


def cpu_host():
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def cpu_baseline(sysm, args, W):
    """The FP64 C oracle, single-threaded, on a bounded sample of the
    workload from its initial state: the first steps of the fixed-margin
    schedule (its first, synchronous detection included; 50 steps up to
    2 M spheres, else 30).  The 60 M-sphere bed is sampled as the same
    recipe at 2 M owners (the same lattice, depth, templates, cylinder and
    step on a quarter of the width), since the oracle's plain detection of
    the full bed alone takes many minutes.  Contact buffers are sized from
    the oracle's own count of the first set."""
    import oracle
    samp = sysm
    note = "same workload"
    if args.workload == "config4" and sysm.n_owners > 2_000_000:
        samp = W.config4(seed=0, n_owners=2_000_000)
        note = (f"the same bed recipe at 2 M owners ({samp.n_spheres} spheres: same lattice, depth, templates, "
                f"cylinder and step, a quarter of the width)")
    o = oracle.Oracle(samp)
    st = o.state()
    Ns = samp.n_spheres
    steps = args.cpu_steps or (50 if Ns <= 2_000_000 else 30)
    n0 = o.detect(st, samp.margin).size
    cap = 4 * n0 + 4096
    while True:
        st = o.state()
        t0 = time.perf_counter()
        try:
            o.run(st, steps, mode="fixed", k=args.k, lam=args.lam, cap=cap)
        except RuntimeError:
            cap *= 2
            continue
        dt = time.perf_counter() - t0
        break
    rate = Ns * steps / dt
    out = {"value": round(rate, 1), "unit": "sphere-steps/s", "cores": 1, "kind": "oracle",
           "sample": (f"{note}: the first {steps} steps of the fixed-margin schedule (k={args.k}) "
                      f"from the initial state, single-threaded FP64 C oracle, {dt:.1f} s")}
    out.update(cpu_host())
    print(f"# cpu oracle: {rate:.4g} sphere-steps/s ({dt:.1f} s)", file=sys.stderr, flush=True)
    return out


def config0_side_by_side(dem, torch, W, steps=2000):
    """The 1,000-sphere case (every-step detection, FP64 oracle next to the
    GPU), timed in full on both sides from the same initial state."""
    import oracle
    s = W.config0(seed=0)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    ctx.step(5)
    ctx.set_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    g = ctx.get_state()
    ctx.close()
    o = oracle.Oracle(s)
    st = o.state()
    t0 = time.perf_counter()
    st, _, stats, _ = o.run(st, steps, mode="every")
    t_orc = time.perf_counter() - t0
    dz = float(np.abs(np.mean(g["X"][:, 2]) - np.mean(st["X"][:, 2])))
    out = {"workload": "1000 spheres r = 5 mm, 10^3 jittered lattice in a 0.2 m box, dt 1e-5 s, "
                       f"every-step detection, {steps} steps",
           "gpu_sphere_steps_per_s": round(s.n_spheres * steps / t_gpu, 1), "gpu_s": round(t_gpu, 3),
           "oracle_sphere_steps_per_s": round(s.n_spheres * steps / t_orc, 1), "oracle_s": round(t_orc, 2),
           "oracle_cores": 1, "mean_height_diff_m": dz}
    print(f"# config0: gpu {out['gpu_sphere_steps_per_s']:.4g}, oracle {out['oracle_sphere_steps_per_s']:.4g} "
          f"sphere-steps/s", file=sys.stderr, flush=True)
    return out


def workload_text(args, Ns, No, n_tri, n_dormant, head):
    lam = args.lam
    if args.workload == "config4":
        return (f"{Ns} spheres in {No} owners on a 7 mm lattice in a 2 x 2 m container (18 of every 32 owners "
                f"single spheres r = 2 mm, the rest tri-sphere clumps r = 2 mm), an analytic cylinder R = 0.1 m, "
                f"L = 0.5 m rolling across the top at 0.2 m/s; dt 5e-6 s, margin 0.2 mm; delayed CD on a second "
                f"HIP stream, adoption latency {lam}; {head} schedule")
    if args.workload == "config1":
        return (f"{Ns} polydisperse spheres r~U(2,3) mm settling from a jittered 7.5 mm lattice in a 0.6x0.6x1.2 m "
                f"box, dt 5e-6 s, margin 0.2 mm, delayed CD on a second HIP stream (adoption latency {lam}); "
                f"{head} schedule")
    if args.workload == "mixer":
        return (f"{Ns} spheres r~U(3,3.5) mm in a bed around a {n_tri}-facet bladed impeller (radius 0.49 m) "
                f"turning at 2 pi rad/s in a 1x1 m box chamber, dt 5e-7 s, margin 0.3 mm, delayed CD on a second "
                f"HIP stream (adoption latency {lam}); {head} schedule")
    if args.workload == "activebox":
        return (f"{Ns} spheres in {No} owners (45 % single r = 2 mm, the rest tri-sphere clumps) on a 7 mm "
                f"lattice in a 1 x 1 m bed, an analytic cylinder rolling on top at 0.2 m/s, dt 5e-6 s, margin "
                f"0.2 mm; active box of 0.5 x 0.6 x 0.1 m around the cylinder ({No - n_dormant} active "
                f"owners), the rest dormant; delayed CD on a second HIP stream; {head} schedule")
    return f"{args.workload}: {Ns} spheres, {No} owners; {head} schedule"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one GPU only (no multi-GPU sharding is implemented); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_2311_04648_amd as dem
    import workloads as W

    if args.copy_probe:
        # a plain copy kernel of known size, for scaling the HBM byte counters
        n = args.copy_probe // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": 4 * n, "reads": 4 * n, "writes": 4 * n, "launches": 5}))
        return

    if not os.path.exists(dem.LIB_PATH):
        from paper_2311_04648_amd import build
        build.build()
    torch.cuda.init()
    if args.timing <= 0:
        args.timing = max(1, min(32, args.steps // 4))
    t_gen = time.perf_counter()
    gens = {"config1": lambda: W.config1(seed=0, n=args.n), "config2": lambda: W.config2(seed=0),
            "config3": lambda: W.config3(seed=7), "config4": lambda: W.config4(seed=0),
            "mixer": lambda: W.mixer(seed=0), "activebox": lambda: W.activebox(seed=0)}
    if args.workload not in gens:
        raise SystemExit(f"unknown workload {args.workload}")
    sysm = gens[args.workload]()
    print(f"# workload generated: {sysm.n_spheres} spheres in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    Ns, No = sysm.n_spheres, sysm.n_owners
    mlp = None
    mlp_safety = 1.0
    mlp_path = os.path.join(ROOT, "paper_2311_04648_amd", "mlp_interval.json")
    if os.path.exists(mlp_path):
        md = json.load(open(mlp_path))
        mlp = np.array(md["params"], dtype=np.float32)
        mlp_safety = float(md.get("safety", 1.0))
    args.mlp_safety = mlp_safety

    modes = [m for m in args.modes.split(",") if m]
    if not args.no_prime:
        t0 = time.perf_counter()
        prime(dem, torch, W, sysm, modes, args, mlp)
        print(f"# primed every schedule on a small system in {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)
    results = {}
    head = "learned" if "learned" in modes else ("fixed" if "fixed" in modes else modes[0])
    for mode in modes:
        r = run_mode(dem, torch, sysm, mode, args, mlp=mlp, turning=mode == head and Ns != No)
        st = r["stats"]
        rate = Ns * args.steps / r["seconds"]
        results[mode] = r
        print(f"# {mode}: {rate:.4g} sphere-steps/s, {1e3 * r['seconds'] / args.steps:.4f} ms/step, "
              f"cds {st['cds']}, mean interval {st['mean_interval']:.1f}, mean set {st['mean_contacts']:.0f}, "
              f"stage ms {['%.2f' % x for x in st['stage_ms']]} n {st['stage_n']}",
              file=sys.stderr, flush=True)
    misses = {}
    if not args.no_judge:
        for mode in modes:
            if mode == "every":
                misses[mode] = 0
                continue
            ctx = make_ctx(dem, sysm, mode, args, mlp, True)
            ctx.set_state()
            st = ctx.step(args.warmup + args.steps)
            misses[mode] = int(st["misses"])
            ctx.close()
            print(f"# judged {mode}: misses {st['misses']} repairs {st['repairs']}", file=sys.stderr, flush=True)

    r = results[head]
    st = r["stats"]
    value = Ns * args.steps / r["seconds"]
    n_clump = int(np.sum(np.asarray(sysm.own_tmpl) >= 0))
    n_tri = int(getattr(sysm, "n_tri", 0))
    fam = np.asarray(getattr(sysm, "owner_family", np.zeros(0)))
    dormant = (np.asarray(sysm.fam_fixed)[fam] > 0) if fam.size else np.zeros(No, dtype=bool)
    n_dormant = int(dormant.sum())
    n_dormant_clump = int(np.sum(dormant & (np.asarray(sysm.own_tmpl) >= 0)))
    n_dormant_sph = int(np.sum(dormant[np.asarray(sysm.sph_owner)])) if n_dormant else 0
    rolling = bool(np.any(np.asarray(sysm.mat_crr) > 0))
    passes = 1   # one-pass bin sort (the LSD radix option would take (sort_bits + 7) // 8)
    # the dynamics form the timed run used: the split clump step (streaming
    # kernel + kernel over the owners with contacts) times its two kernels as
    # stages 1 and 0; the fused step times runs of launches as stage 1; the
    # two-kernel form its force and fold kernels as stages 0 and 1
    tot, cnt = st["stage_ms"], st["stage_n"]
    split = args.dyn_path != 1 and int(cnt[0]) > 0
    if args.dyn_path == 1:
        names = ["k_force", "k_fold_integrate"]
    elif split:
        names = ["k_step_listed", "k_step_free"]
    else:
        names = ["k_force", "k_step_fused"]
    dom = 0 if tot[0] > tot[1] else 1
    n_launch = max(int(cnt[dom]), 1)
    avg_raw = tot[dom] / n_launch
    # every event pair around the dynamics kernel(s) is followed by an empty
    # one-wave kernel bracketed the same way: its interval is the markers'
    # own overhead, paid once per pair
    n_noop = max(int(cnt[4]), 1)
    stamp_ms = tot[4] / n_noop
    pairs_dom = n_launch if (split or args.dyn_path == 1) else n_noop
    avg_ms = max((tot[dom] - stamp_ms * pairs_dom) / n_launch, 1e-6)
    C = st["mean_contacts"]
    # (the split clump step moves the orientation of turning clumps only)
    n_clump_q = r["n_turn"] if (split and r["n_turn"] is not None) else n_clump
    kw = dict(clumps=Ns != No, rolling=rolling, n_clump=n_clump_q, n_tri=n_tri, n_dormant=n_dormant,
              n_dormant_clump=min(n_dormant_clump, n_clump_q))
    if split:
        algo_k = {"k_step_free": stream_bytes(No, r["n_turn"] if r["n_turn"] is not None else n_clump, r["n_spin"]),
                  "k_step_listed": listed_bytes(r["active_owners"], n_clump_share(sysm, r), r["active"], C,
                                                rolling)}
    else:
        # (pair skipping: single spheres without fixed families, dense sets)
        keys_on = (Ns == No and n_dormant == 0 and not bool(np.any(np.asarray(sysm.fam_fixed) > 0))
                   and args.dyn_path != 1 and 2 * C >= Ns)
        algo_k = {names[dom]: algorithmic_bytes(names[dom] if names[dom] != "k_force" or args.dyn_path == 1
                                                else "k_step_fused", Ns, No, C, r["active"],
                                                r["info"]["nbins"], passes,
                                                pair_keys=keys_on and names[dom] == "k_step_fused", **kw)}
    algo = algo_k[names[dom]]
    timed = int(cnt[dom]) > 0
    achieved = algo / (avg_ms * 1e-3) / 1e9 if timed else None
    traffic = load_traffic(names[dom], args.workload)
    roofline = {"bound": "hbm", "kernel": names[dom], "achieved": round(achieved, 2) if timed else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if timed else None,
                "traffic": traffic,
                "algorithmic_bytes_per_launch": int(algo), "avg_launch_ms": round(avg_ms, 5) if timed else None,
                "event_interval_per_launch_ms": round(avg_raw, 5), "event_pair_overhead_ms": round(stamp_ms, 5),
                "event_pairs": int(cnt[4]), "launches": n_launch, "sampled_every_steps": args.timing}
    if split:
        other = names[1 - dom]
        n_o = max(int(cnt[1 - dom]), 1)
        o_ms = max((tot[1 - dom] - stamp_ms * n_o) / n_o, 1e-6)
        roofline["second_kernel"] = {"kernel": other, "avg_launch_ms": round(o_ms, 5),
                                     "algorithmic_bytes_per_launch": int(algo_k[other]),
                                     "achieved": round(algo_k[other] / (o_ms * 1e-3) / 1e9, 1)}
    n_cd = max(int(cnt[2]), 1)
    cd_ms = tot[2] / n_cd
    cd_bytes = algorithmic_bytes("detect", Ns, No, C, r["active"], r["info"]["nbins"], passes, n_tri=n_tri,
                                 n_dormant_sph=n_dormant_sph)
    cd_chain = {"avg_ms": round(cd_ms, 4), "launches": n_cd, "algorithmic_bytes": int(cd_bytes),
                "achieved_GBs": round(cd_bytes / (cd_ms * 1e-3) / 1e9, 1) if cd_ms > 0 else None,
                "note": "detection chain on the second stream, concurrent with the dynamics stream"}

    cpu = None
    if not args.no_cpu and n_tri == 0 and n_dormant == 0:
        cpu = cpu_baseline(sysm, args, W)
    c0 = None
    if not args.no_config0:
        c0 = config0_side_by_side(dem, torch, W)

    # measured streaming bandwidth of a plain device copy (2 x 1 GiB moved per copy)
    nb = 1 << 28
    src = torch.ones(nb, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(10):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    copy_gbs = 2 * 4 * nb / (sorted(times)[len(times) // 2] * 1e-3) / 1e9
    del src, dst
    roofline["measured_copy_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbs, 4) if timed else None

    # single-sphere runs without fixed families: a delayed work order's
    # binning step rides on the step kernel, which reads the state anyway
    fused_front = (Ns == No and not bool(np.any(np.asarray(sysm.fam_fixed) > 0)) and args.dyn_path != 1)

    def skip_keys(C):
        # pair skipping runs in the staged step of single-sphere systems
        # without fixed families: dense sets (one contact per two spheres)
        return fused_front and 2 * C >= Ns

    def path_bytes_per_step(rr, mode):
        # algorithmic bytes of one step of the whole path: the dynamics
        # kernel(s) every step, detection once per detection, and the remap
        # pass once per detection in the two-kernel form (the step right
        # after an adoption carries the history over itself, reading it for
        # touching pairs only)
        s2 = rr["stats"]
        Cm, act = s2["mean_contacts"], rr["active"]
        if args.dyn_path != 1:
            dyn_b = algorithmic_bytes("k_step_fused", Ns, No, Cm, act, 0, passes, pair_keys=skip_keys(Cm), **kw)
        else:
            dyn_b = (algorithmic_bytes("k_force", Ns, No, Cm, act, 0, passes)
                     + algorithmic_bytes("k_fold_integrate", Ns, No, Cm, act, 0, passes, clumps=Ns != No))
        per_cd = algorithmic_bytes("detect", Ns, No, Cm, act, rr["info"]["nbins"], passes, n_tri=n_tri,
                                   n_dormant_sph=n_dormant_sph)
        if fused_front and mode not in ("every", "adaptive"):
            per_cd -= 64 * (Ns - n_dormant_sph)   # (the sphere and owner records are not read a second time)
        if args.dyn_path == 1:
            per_cd += algorithmic_bytes("k_remap", Ns, No, Cm, act, 0, passes)
        return dyn_b + per_cd * s2["cds"] / args.steps

    modes_out = {}
    for mode, rr in results.items():
        s2 = rr["stats"]
        bps = path_bytes_per_step(rr, mode)
        gbs = bps / (rr["seconds"] / args.steps) / 1e9
        modes_out[mode] = {"value": round(Ns * args.steps / rr["seconds"], 1),
                           "ms_per_step": round(1e3 * rr["seconds"] / args.steps, 5),
                           "algorithmic_bytes_per_step": int(bps), "achieved_GBs": round(gbs, 1),
                           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "copy_frac": round(gbs / copy_gbs, 4),
                           "cds": int(s2["cds"]), "mean_interval": round(s2["mean_interval"], 2),
                           "mean_contacts": round(s2["mean_contacts"], 1),
                           "missed_contacts": misses.get(mode),
                           "stage_ms": [round(x, 3) for x in s2["stage_ms"]],
                           "stage_launches": [int(x) for x in s2["stage_n"]]}
    out = {
        "metric": "sphere-steps/s (CD+force+integrate) at 1 GPU; learned vs fixed-margin CD",
        "value": round(value, 1),
        "unit": "sphere-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["seconds"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload_text(args, Ns, No, n_tri, n_dormant, head),
                   "n_spheres": Ns, "n_owners": No, "schedule": head, "k": args.k, "lambda": args.lam,
                   "dynamics": ("streaming kernel + kernel over the owners with contacts" if split else
                                "one fused kernel per step" if args.dyn_path != 1 else "force + fold kernels")},
        "modes": modes_out,
        "missed_contacts": misses.get(head),
        "roofline": roofline,
        "cd_chain": cd_chain,
        "cpu_baseline": cpu,
        "config0_side_by_side": c0,
    }
    if "fixed" in results and head != "fixed":
        out["vs_fixed"] = round(value / modes_out["fixed"]["value"], 4)
    if n_dormant:
        act_sph = int(np.sum(~dormant[np.asarray(sysm.sph_owner)]))
        out["config"]["active_owners"] = No - n_dormant
        out["config"]["active_spheres"] = act_sph
        out["active_sphere_steps_per_s"] = round(act_sph * args.steps / r["seconds"], 1)
        out["value_note"] = "nominal: all spheres counted, the dormant ones included (as the paper counts its rover run)"
        # the same bed and schedule with every owner active, for comparison
        import copy
        full = copy.copy(sysm)
        full.owner_family = np.zeros(0, dtype=np.uint8)
        full.fam_pair_off = np.zeros(0, dtype=np.uint8)
        full.fam_fixed = np.zeros(0, dtype=np.uint8)
        full.V = np.zeros_like(sysm.V)
        full.W = np.zeros_like(sysm.W)
        rf = run_mode(dem, torch, full, head, args, mlp=mlp)
        out["full_domain"] = {"value": round(Ns * args.steps / rf["seconds"], 1),
                              "ms_per_step": round(1e3 * rf["seconds"] / args.steps, 5),
                              "mean_contacts": round(rf["stats"]["mean_contacts"], 1)}
        print(f"# full domain ({head}): {Ns * args.steps / rf['seconds']:.4g} sphere-steps/s", file=sys.stderr,
              flush=True)
    if n_tri:
        out["config"]["n_facets"] = n_tri
        # the paper's own mixer figure, for context only (2 A100s, its own
        # 2892-facet mesh after 1 s of mixing): 0.546 h per 1e6 steps per 1e6 spheres
        out["paper_mixer_sphere_steps_per_s"] = 5.09e8
        out["cpu_baseline_note"] = ("not run for this workload: the oracle tests every facet against every "
                                    "sphere (about 3e9 closest-point tests per detection at this size)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
