"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (derived from the arithmetic, see the design notes):
  * contact pair sets: bit-exact (both sides evaluate the same FP64 predicate
    on the same exact sphere centres);
  * per-contact force / torque: |F_gpu - F_orc| <= 1e-5 max(|F_orc|, 1e-3 F_med)
    (FP32 force law, FP64 overlap);
  * one-step increments: |d_gpu - d_orc| <= 1e-5 |d_orc| + a storage floor:
    X on a 2^-38 m grid, velocities stored in FP32 (half an ulp of the new
    value) plus 1e-5 of the summed contact-force magnitudes of the owner
    (reductions of cancelling terms).
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dem():
    import paper_2311_04648_amd as d
    if not os.path.exists(d.LIB_PATH):
        from paper_2311_04648_amd import build
        build.build()
    d._torch()
    return d


def cluster(n_small=60, R=0.006, r=0.0015):
    """One large sphere with small ones on its surface: rows far longer than
    the 16 staged partners of the single-traversal detection."""
    k = np.arange(n_small) + 0.5
    phi = np.arccos(1 - 2 * k / n_small)
    th = np.pi * (1 + 5 ** 0.5) * k
    d = R + r - 2e-5
    pts = d * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    X = np.vstack([np.zeros((1, 3)), pts])
    rad = np.r_[R, np.full(n_small, r)]
    rng = np.random.default_rng(0)
    V = rng.normal(0, 0.05, size=X.shape)
    return W.assemble(np.full(X.shape[0], -1), X, W._qid(X.shape[0]), V, np.zeros_like(X), [], rad, None,
                      W.box_walls(-0.02 * np.ones(3), 0.02 * np.ones(3)), W.materials(), (0, 0, -9.81), 2e-6,
                      0.0002, -0.02 * np.ones(3), 0.02 * np.ones(3), name="cluster")


def systems():
    return {
        "cluster": cluster(),
        "spheres": W.small_spheres(1, n=343),
        "clumps": W.small_clumps(2, n=150, with_cylinder=True, spacing=0.0085),
        "config0": W.config0(),
        "spheres_ragged": W.small_spheres(3, n=1001, r=(0.0015, 0.004)),
    }


SYS = systems()


def _gpu_state(ctx):
    g = ctx.get_state()
    return {k: np.asarray(g[k], dtype=np.float64) for k in ("X", "q", "V", "W")}, g["step"]


def _world_w(s, st):
    """Angular velocity in the world frame (oracle layout: body frame + q)."""
    from scipy.spatial.transform import Rotation
    R = Rotation.from_quat(st["q"][:, [1, 2, 3, 0]]).as_matrix()
    return np.einsum("nij,nj->ni", R, st["W"])


def _gpu_world_w(s, g):
    w = np.asarray(g["W"], dtype=np.float64)
    clump = s.own_tmpl >= 0
    if clump.any():
        from scipy.spatial.transform import Rotation
        R = Rotation.from_quat(g["q"][clump][:, [1, 2, 3, 0]]).as_matrix()
        w[clump] = np.einsum("nij,nj->ni", R, w[clump])
    return w


def _orc_state_from_gpu(s, g):
    """The oracle takes the GPU's stored state; single spheres carry their
    world-frame angular velocity with q = identity."""
    return {"X": g["X"].copy(), "q": g["q"].copy(), "V": g["V"].astype(np.float64),
            "W": g["W"].astype(np.float64)}


@pytest.mark.parametrize("name", list(SYS))
def test_state_roundtrip_exact(dem, name):
    s = SYS[name]
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    g = ctx.get_state()
    np.testing.assert_array_equal(g["X"], s.X)
    np.testing.assert_array_equal(g["V"], s.V.astype(np.float32))
    clump = s.own_tmpl >= 0
    np.testing.assert_array_equal(g["q"][clump], s.q[clump])


@pytest.mark.parametrize("name", list(SYS))
@pytest.mark.parametrize("bin_sort", [0, 1])
def test_binning_sort_is_stable_permutation(dem, name, bin_sort):
    s = SYS[name]
    ctx = dem.DemContext(s, mode="every", bin_sort=bin_sort)
    ctx.set_state()
    keys, ids = ctx.bin()
    assert np.all(np.diff(keys.astype(np.int64)) >= 0)
    assert np.array_equal(np.sort(ids), np.arange(s.n_spheres))
    same = np.diff(keys.astype(np.int64)) == 0
    assert np.all(np.diff(ids.astype(np.int64))[same] > 0)
    # the one-pass bin sort and the LSD radix sort give the same order,
    # equal to numpy's stable argsort of the keys
    other = dem.DemContext(s, mode="every", bin_sort=1 - bin_sort)
    other.set_state()
    k2, i2 = other.bin()
    np.testing.assert_array_equal(keys, k2)
    np.testing.assert_array_equal(ids, i2)
    order = np.argsort(keys[np.argsort(ids)], kind="stable")
    np.testing.assert_array_equal(ids, order.astype(np.uint32))


@pytest.mark.parametrize("name", list(SYS))
@pytest.mark.parametrize("margin_scale", [0.0, 1.0])
def test_contact_sets_bit_exact(dem, name, margin_scale):
    s = SYS[name]
    m = margin_scale * (s.margin if s.margin > 0 else 0.001)
    ctx = dem.DemContext(s, mode="fixed", margin=max(m, 1e-4))
    ctx.set_state()
    n = ctx.detect_contacts(m)
    keys, hist = ctx.get_contacts()
    assert n == keys.size
    o = oracle.Oracle(s)
    ref = o.detect(o.state(), m)
    assert ref.size > 0 or (name == "config0" and m == 0.0)
    np.testing.assert_array_equal(keys, ref)
    assert np.all(hist == 0)


def _force_case(dem, s, seed=0, presteps=0, ages=False):
    ctx = dem.DemContext(s, mode="fixed", margin=max(s.margin, 1e-4))
    ctx.set_state()
    if presteps:
        ctx.step(presteps)
    ctx.detect_contacts(max(s.margin, 1e-4))
    keys, _ = ctx.get_contacts()
    rng = np.random.default_rng(seed)
    hist = W.f32(rng.normal(0.0, 3e-6, size=(keys.size, 4))).astype(np.float32)
    hist[:, 3] = W.f32(rng.uniform(0.0, 3e-5, size=keys.size)) if ages else 0.0
    ctx.set_contacts(keys, hist)
    ctx.forces()
    Fo, To, Fc = ctx.get_forces(keys.size)
    k2, h2 = ctx.get_contacts()
    g = ctx.get_state()
    o = oracle.Oracle(s)
    ost = _orc_state_from_gpu(s, g)
    ref = o.forces(ost, keys, hist.astype(np.float64), step=g["step"])
    _force_case.last = (ost, hist, g["step"])
    return keys, Fo, To, Fc, h2, ref


@pytest.mark.parametrize("name", list(SYS))
def test_forces_match_oracle(dem, name):
    s = SYS[name]
    keys, Fo, To, Fc, h2, ref = _force_case(dem, s, presteps=1500 if name == "config0" else 0)
    touch = ref["touch"] > 0
    assert touch.sum() > 10
    Fn = np.linalg.norm(ref["Fc"], axis=1)
    Fmed = np.median(Fn[touch])
    err = np.linalg.norm(Fc - ref["Fc"], axis=1)
    rel = err / np.maximum(Fn, 1e-3 * Fmed)
    print(f"{name}: contacts {keys.size} touching {touch.sum()} max rel F err {rel.max():.2e} "
          f"median {np.median(rel[touch]):.2e}")
    assert rel.max() <= 1e-5
    # false positives: exactly zero force and released history
    assert np.all(Fc[~touch] == 0.0)
    assert np.all(h2[~touch] == 0.0)
    # history
    hn = np.linalg.norm(ref["hist"][:, :3], axis=1)
    hmed = np.median(hn[touch]) if touch.any() else 1.0
    herr = np.linalg.norm(h2[:, :3] - ref["hist"][:, :3], axis=1) / np.maximum(hn, 1e-3 * hmed)
    assert herr.max() <= 1e-5
    # owner sums: tolerance relative to the summed magnitudes of the terms
    own = s.sph_owner
    ks = (keys >> np.uint64(32)).astype(np.int64)
    L1 = np.zeros(s.n_owners)
    np.add.at(L1, own[ks], Fn)
    js = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    sph = js < s.n_spheres
    np.add.at(L1, own[js[sph]], Fn[sph])
    ferr = np.linalg.norm(Fo - ref["Fo"], axis=1)
    assert np.all(ferr <= 1e-5 * np.maximum(L1, 1e-3 * Fmed) + 1e-30)
    terr = np.linalg.norm(To - ref["To"], axis=1)
    Tscale = L1 * 0.006
    assert np.all(terr <= 1e-5 * np.maximum(Tscale, 1e-3 * Fmed * 0.003) + 1e-30)


def test_rolling_resistance_matches_oracle(dem):
    """Default model with C_rr > 0: the torque-only rolling-resistance force
    and the contact-age gate (Eq. (2), default-model walk-through)."""
    s = W.small_spheres(21, n=343, vel=0.3)
    s.mat_crr[:] = 0.1
    keys, Fo, To, Fc, h2, ref = _force_case(dem, s, seed=4, ages=True)
    touch = ref["touch"] > 0
    assert touch.sum() > 10
    Fn = np.linalg.norm(ref["Fc"], axis=1)
    Fmed = np.median(Fn[touch])
    rel = np.linalg.norm(Fc - ref["Fc"], axis=1) / np.maximum(Fn, 1e-3 * Fmed)
    assert rel.max() <= 1e-5
    np.testing.assert_allclose(h2[touch, 3], ref["hist"][touch, 3], rtol=1e-6)
    assert np.all(h2[~touch, 3] == 0.0)
    L1 = np.zeros(s.n_owners)
    ks = (keys >> np.uint64(32)).astype(np.int64)
    js = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.add.at(L1, s.sph_owner[ks], Fn)
    sph = js < s.n_spheres
    np.add.at(L1, s.sph_owner[js[sph]], Fn[sph])
    terr = np.linalg.norm(To - ref["To"], axis=1)
    assert np.all(terr <= 1e-5 * np.maximum(L1 * 0.006, 1e-3 * Fmed * 0.003) + 1e-30)
    # the rolling torque is on: torques differ from the C_rr = 0 model
    ost, hist, step = _force_case.last
    s0 = W.small_spheres(21, n=343, vel=0.3)
    ref0 = oracle.Oracle(s0).forces(ost, keys, hist.astype(np.float64), step=step)
    assert np.abs(ref["To"] - ref0["To"]).max() > 1e-3 * np.abs(ref["To"]).max()


@pytest.mark.parametrize("name", list(SYS) + ["rolling"])
def test_one_step_matches_oracle(dem, name):
    if name == "rolling":
        s = W.small_spheres(22, n=343, vel=0.3)
        s.mat_crr[:] = 0.1
    else:
        s = SYS[name]
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    g0 = ctx.get_state()
    st = _orc_state_from_gpu(s, g0)
    ctx.step(1)
    g1 = ctx.get_state()
    o = oracle.Oracle(s)
    before = {k: v.copy() for k, v in st.items()}
    st1, acs, stats, _ = o.run(st, 1, mode="every")
    keys = acs[0]
    # per-owner L1 norm of contact forces (tolerance floor for sums)
    out = o.forces(before, keys, np.zeros((keys.size, 3)))
    Fn = np.linalg.norm(out["Fc"], axis=1)
    L1 = np.zeros(s.n_owners)
    ks = (keys >> np.uint64(32)).astype(np.int64)
    js = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.add.at(L1, s.sph_owner[ks], Fn)
    sph = js < s.n_spheres
    np.add.at(L1, s.sph_owner[js[sph]], Fn[sph])
    h = s.dt
    # velocity
    dv_g = g1["V"].astype(np.float64) - before["V"]
    dv_o = st1["V"] - before["V"]
    tol_v = 1e-5 * np.linalg.norm(dv_o, axis=1) + 0.5 * np.spacing(np.abs(g1["V"]).max(1).astype(np.float32)) \
        * 2 + 1e-5 * h * L1 / s.own_mass
    assert np.all(np.linalg.norm(dv_g - dv_o, axis=1) <= tol_v)
    # position
    dx_g = g1["X"] - before["X"]
    dx_o = st1["X"] - before["X"]
    tol_x = 1e-5 * np.linalg.norm(dx_o, axis=1) + h * np.linalg.norm(dv_g - dv_o, axis=1) + 2.0 ** -37
    assert np.all(np.linalg.norm(dx_g - dx_o, axis=1) <= tol_x)
    # angular velocity (world frame)
    w0 = _world_w(s, before)
    wg = _gpu_world_w(s, g1)
    wo = _world_w(s, st1)
    dw_g, dw_o = wg - w0, wo - w0
    Iinv = 1.0 / s.own_moi.min(1)
    tol_w = 1e-5 * np.linalg.norm(dw_o, axis=1) + 4 * np.spacing(np.abs(wg).max(1).astype(np.float32)) \
        + 1e-5 * h * L1 * 0.01 * Iinv
    assert np.all(np.linalg.norm(dw_g - dw_o, axis=1) <= tol_w)
    clump = s.own_tmpl >= 0
    if clump.any():
        dq_g = g1["q"][clump] - before["q"][clump]
        dq_o = st1["q"][clump] - before["q"][clump]
        tol_q = 1e-5 * np.linalg.norm(dq_o, axis=1) + h * np.linalg.norm(dw_g - dw_o, axis=1)[clump] + 1e-15
        assert np.all(np.linalg.norm(dq_g - dq_o, axis=1) <= tol_q)


def _fused_case(name):
    if name == "rolling":
        s = W.small_spheres(23, n=512, vel=0.3)
        s.mat_crr[:] = 0.1
        return s
    if name == "clumps_dense":
        return W.small_clumps(6, n=300, vel=0.3, with_cylinder=True, spacing=0.0080)
    if name == "wide_margin":
        return wide_margin_lattice()
    return SYS[name]


def wide_margin_lattice(m=10, r=0.001, gap=5e-5, margin=0.0015):
    """A cubic lattice of nearly touching spheres with a margin of 1.5
    radii: about 20 pairs per sphere in the set, so the rows of 64
    consecutive spheres hold far more than one wave's LDS slice of
    history (512 entries) and the fused step stages part of them."""
    g = np.arange(m) * (2 * r + gap)
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)[:, ::-1].copy()
    X -= X.mean(0)
    n = X.shape[0]
    rng = np.random.default_rng(4)
    V = rng.normal(0, 0.05, size=X.shape)
    L = 0.02
    return W.assemble(np.full(n, -1), X, W._qid(n), V, np.zeros_like(X), [], r, None,
                      W.box_walls(-L * np.ones(3), L * np.ones(3)), W.materials(), (0, 0, -9.81), 2e-6,
                      margin, -L * np.ones(3), L * np.ones(3), name="wide_margin")


@pytest.mark.parametrize("name", ["cluster", "spheres", "clumps", "clumps_dense", "spheres_ragged", "rolling",
                                  "wide_margin"])
def test_fused_step_equals_two_kernel_path_bitwise(dem, name):
    """The fused step (each owner re-evaluates its B-side contacts with the
    same function) gives the bits of the two-kernel path (per-contact
    reactions written, then the ordered fold): state, contact set and
    history, over a delayed schedule on two streams; with its history
    writes staged per wave in LDS (path 2), not staged (3) and staged as
    the last contact count says (0); and, for clump systems, as a streaming
    kernel plus a kernel over the owners with contacts (4, and 0 when the
    set is sparse)."""
    import torch
    s = _fused_case(name)
    out = []
    for path in (1, 0, 2, 3, 4):
        c = dem.DemContext(s, mode="fixed", k=5, lam=2, dyn_path=path, capacity=64 * s.n_spheres)
        c.set_state()
        c.step(120, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
        g = c.get_state()
        keys, hist = c.get_contacts()
        out.append((g, keys, hist))
        c.close()
    ga, ka, ha = out[0]
    assert ka.size > 0
    if name == "wide_margin":
        assert ka.size > 15 * s.n_spheres
    for gb, kb, hb in out[1:]:
        for k in ("X", "V", "W", "q"):
            np.testing.assert_array_equal(ga[k], gb[k])
        np.testing.assert_array_equal(ka, kb)
        np.testing.assert_array_equal(ha, hb)


def test_delayed_equals_every_step_bitwise(dem):
    """Sec. 2.1: delayed detection with a sufficient margin reproduces the
    every-step trajectory exactly (false positives add exact zeros, the
    per-owner fold runs in a fixed order)."""
    s = W.small_spheres(5, n=512, vel=0.3)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(200)
    b = dem.DemContext(s, mode="fixed", k=10, lam=5, judge=True)
    b.set_state()
    stats = b.step(200)
    assert stats["misses"] == 0 and stats["cds"] == 20
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])


def test_delayed_two_streams_equals_every_step_bitwise(dem):
    import torch
    s = W.small_clumps(6, n=216, vel=0.3)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(150)
    b = dem.DemContext(s, mode="fixed", k=8, lam=4)
    b.set_state()
    dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
    b.step(150, dyn=dyn, kin=kin)
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("judge", [False, True])
def test_zero_latency_schedule_equals_every_step_bitwise(dem, streams, judge):
    """Sec. 2.1 with no delay (lambda = 0): each set is adopted at the step
    of its own work order, so that step must run on the new set; the
    trajectory equals every-step detection bit for bit (single spheres,
    where a work order's binning may otherwise ride on the step kernel)."""
    import torch
    s = W.small_spheres(5, n=512, vel=0.3)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(120)
    b = dem.DemContext(s, mode="fixed", k=10, lam=0, judge=judge)
    b.set_state()
    if streams == 2:
        dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
        stats = b.step(120, dyn=dyn, kin=kin)
    else:
        stats = b.step(120)
    assert stats["cds"] == 12 and stats["swaps"] == 12
    if judge:
        assert stats["misses"] == 0
    assert stats["mean_contacts"] > 0
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])
    ka, ha = a.get_contacts()
    kb, hb = b.get_contacts()
    assert np.array_equal(np.intersect1d(ka, kb), ka)


@pytest.mark.parametrize("streams", [1, 2])
def test_adaptive_schedule_equals_every_step_bitwise(dem, streams):
    """Sec. 2.1's own policy (work order at every adoption, latency adapted
    from timing, margin from n_max = 2 lambda): judged, no contact is
    missed, and the trajectory equals every-step detection bit for bit."""
    import torch
    s = W.small_spheres(5, n=512, vel=0.3)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(300)
    b = dem.DemContext(s, mode="adaptive", k=10, lam=2, judge=True, k_max=64)
    b.set_state()
    kw = dict(dyn=torch.cuda.Stream(), kin=torch.cuda.Stream()) if streams == 2 else {}
    stats = b.step(300, **kw)
    assert stats["misses"] == 0
    assert stats["cds"] > 300 // 64
    assert 1.0 <= stats["mean_interval"] <= 64.0
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])


def test_adaptive_schedule_with_binding_margin_cap_stays_exact(dem):
    """A run margin far below what n_max needs: the derived margin is capped,
    the latency shrinks, the judge repairs what the small margin misses, and
    the trajectory still equals every-step detection."""
    s = W.small_spheres(6, n=343, vel=1.0)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(200)
    b = dem.DemContext(s, mode="adaptive", k=10, lam=4, judge=True, margin=2e-6, k_max=64)
    b.set_state()
    stats = b.step(200)
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])
    assert stats["cds"] >= 200 // 8


def test_judge_counts_misses_and_repair_restores_exactness(dem):
    s = W.small_spheres(7, n=343, vel=1.0, margin=1e-6)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(120)
    b = dem.DemContext(s, mode="fixed", k=30, lam=10, judge=True, repair=True)
    b.set_state()
    stats = b.step(120)
    assert stats["misses"] > 0 and stats["repairs"] > 0
    ga, gb = a.get_state(), b.get_state()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])


def test_judge_without_repair_reports_missed(dem):
    s = W.small_spheres(7, n=343, vel=1.0, margin=1e-6)
    b = dem.DemContext(s, mode="fixed", k=30, lam=10, judge=True, repair=False)
    b.set_state()
    with pytest.raises(dem.DemError) as e:
        b.step(120)
    assert e.value.status == dem.DEM_ERR_MISSED


def test_run_is_deterministic(dem):
    s = W.small_clumps(8, n=216, vel=0.5)
    outs = []
    for _ in range(2):
        c = dem.DemContext(s, mode="fixed", k=10, lam=3)
        c.set_state()
        c.step(100)
        outs.append(c.get_state())
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])


def test_resume_from_checkpoint_is_bitwise(dem):
    s = W.small_spheres(9, n=343, vel=0.3)
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(60)
    b = dem.DemContext(s, mode="every")
    b.set_state()
    b.step(30)
    g = b.get_state()
    keys, hist = b.get_contacts()
    c = dem.DemContext(s, mode="every")
    c.set_state(g["X"], g["q"], g["V"], g["W"], step=g["step"])
    c.set_contacts(keys, hist)
    c.step(30)
    ga, gc = a.get_state(), c.get_state()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(ga[k], gc[k])


def test_capacity_error_reports_required_size(dem):
    s = W.small_spheres(1, n=343)
    ctx = dem.DemContext(s, mode="every", capacity=20)
    ctx.set_state()
    with pytest.raises(dem.DemError) as e:
        ctx.detect_contacts(0.0)
    assert e.value.status == dem.DEM_ERR_CAPACITY
    need = e.value.required
    o = oracle.Oracle(s)
    assert need == o.detect(o.state(), 0.0).size
    ctx.bind(need + 10)
    ctx.set_state()
    assert ctx.detect_contacts(0.0) == need


@pytest.mark.parametrize("dyn_path", [0, 1])
def test_capacity_overflow_during_steps_stops(dem, dyn_path):
    s = W.small_spheres(1, n=343)
    ctx = dem.DemContext(s, mode="every", capacity=20, dyn_path=dyn_path)
    ctx.set_state()
    with pytest.raises(dem.DemError) as e:
        ctx.step(5)
    assert e.value.status == dem.DEM_ERR_CAPACITY
    g = ctx.get_state()
    np.testing.assert_array_equal(g["X"], s.X)


@pytest.mark.parametrize("dyn_path", [0, 1])
def test_divergence_guard(dem, dyn_path):
    s = W.small_spheres(1, n=343, vel=0.5)
    ctx = dem.DemContext(s, mode="every", v_error_out=0.05, dyn_path=dyn_path)
    ctx.set_state()
    with pytest.raises(dem.DemError) as e:
        ctx.step(5)
    assert e.value.status == dem.DEM_ERR_DIVERGED


@pytest.mark.parametrize("dyn_path", [3, 4])
def test_divergence_guard_clumps(dem, dyn_path):
    """Clump systems: a run that diverges stops with DEM_ERR_DIVERGED, and
    every later step of the call copies the state unchanged, with one fused
    kernel (3) and with the streaming kernel plus the kernel over the owners
    with contacts (4): the two end in the same state."""
    s = W.small_clumps(3, n=216, vel=0.5)
    out = []
    for p in (1, dyn_path):
        ctx = dem.DemContext(s, mode="fixed", k=4, lam=2, v_error_out=0.05, dyn_path=p)
        ctx.set_state()
        with pytest.raises(dem.DemError) as e:
            ctx.step(9)
        assert e.value.status == dem.DEM_ERR_DIVERGED
        out.append(ctx.get_state())
        ctx.close()
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


@pytest.mark.parametrize("dyn_path", [3, 4])
def test_capacity_overflow_during_steps_stops_clumps(dem, dyn_path):
    s = W.small_clumps(1, n=216, spacing=0.0085)
    o = oracle.Oracle(s)
    assert o.detect(o.state(), 0.0).size > 20
    ctx = dem.DemContext(s, mode="every", capacity=20, dyn_path=dyn_path)
    ctx.set_state()
    with pytest.raises(dem.DemError) as e:
        ctx.step(5)
    assert e.value.status == dem.DEM_ERR_CAPACITY
    g = ctx.get_state()
    np.testing.assert_array_equal(g["X"], s.X)


def test_resting_clumps_split_step_equals_two_kernel_form(dem):
    """Clumps released at rest, half of them not turning, fall onto the
    floor (strong gravity) and start to turn where they land.  The
    streaming step touches the orientation of a clump at rest neither to
    read nor to write it; the split step must still give the two-kernel
    form's state bit for bit, orientations included, on two streams."""
    import torch
    s = W.small_clumps(12, n=200, vel=0.0, spacing=0.0125, jitter=0.0002, gravity=(0, 0, -200.0))
    s.W[::2] = 0.0
    out = []
    for path in (4, 1):
        c = dem.DemContext(s, mode="fixed", k=10, lam=5, dyn_path=path)
        c.set_state()
        c.step(3000, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
        out.append((c.get_state(), c.get_contacts()[0]))
        c.close()
    (ga, ka), (gb, kb) = out
    for k in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])
    np.testing.assert_array_equal(ka, kb)
    clump = s.own_tmpl >= 0
    turning = np.any(ga["W"] != 0, axis=1)
    print(f"{ka.size} pairs; clumps turning {np.sum(clump & turning)}, at rest {np.sum(clump & ~turning)}",
          flush=True)
    assert ka.size > 20
    assert np.sum(clump & turning) > 0 and np.sum(clump & ~turning) > 0


def test_packed_clumps_split_step_equals_two_kernel_form(dem):
    """Packed clumps (many contacts per owner): the split step's kernel over
    the owners with contacts evaluates an owner's items a few at a time in
    a group of lanes and adds them in order; owners with more items than a
    group has lanes take several rounds.  Bit for bit the two-kernel form,
    on two streams, over a delayed schedule."""
    import torch
    # (a 3 mm margin: every clump lists dozens of pairs with its neighbours)
    s = W.small_clumps(3, n=216, spacing=0.0085, vel=0.02, margin=0.003)
    out = []
    for path in (4, 1):
        c = dem.DemContext(s, mode="fixed", k=5, lam=2, dyn_path=path, capacity=64 * s.n_spheres)
        c.set_state()
        c.step(400, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
        out.append((c.get_state(), c.get_contacts()))
        c.close()
    (ga, (ka, ha)), (gb, (kb, hb)) = out
    for k in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])
    np.testing.assert_array_equal(ka, kb)
    np.testing.assert_array_equal(ha, hb)
    # items per owner: its spheres' row entries and B-list entries
    ki = (ka >> np.uint64(32)).astype(np.int64)
    kj = (ka & np.uint64(0xFFFFFFFF)).astype(np.int64)
    items = np.bincount(s.sph_owner[ki], minlength=s.n_owners)
    sph = kj < s.n_spheres
    items += np.bincount(s.sph_owner[kj[sph]], minlength=s.n_owners)
    print(f"{ka.size} pairs; largest item count of an owner {items.max()}", flush=True)
    assert items.max() > 16


def test_divergence_guard_on_the_delayed_schedule(dem):
    """A run that diverges at its first step under the fixed-margin schedule
    on two streams: the later steps (a work-order step, whose binning rides
    on the halted step, and the first step on the adopted set, which carries
    the history over) copy the state unchanged, and the run ends with the
    state of the every-step run that diverges the same way."""
    import torch
    s = W.small_spheres(1, n=343, vel=0.5)
    out = []
    for mode in ("every", "fixed"):
        ctx = dem.DemContext(s, mode=mode, k=3, lam=1, v_error_out=0.05)
        ctx.set_state()
        kw = dict(dyn=torch.cuda.Stream(), kin=torch.cuda.Stream()) if mode == "fixed" else {}
        with pytest.raises(dem.DemError) as e:
            ctx.step(12, **kw)
        assert e.value.status == dem.DEM_ERR_DIVERGED
        out.append(ctx.get_state())
        ctx.close()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_count_missing_matches_oracle(dem):
    s = W.small_spheres(4, n=343, vel=1.0)
    ctx = dem.DemContext(s, mode="fixed", k=10, lam=0)
    ctx.set_state()
    ctx.detect_contacts(0.0)
    keys0, _ = ctx.get_contacts()
    ctx2 = dem.DemContext(s, mode="every")
    ctx2.set_state()
    ctx2.step(40)
    g = ctx2.get_state()
    ctx.set_state(g["X"], g["q"], g["V"], g["W"], step=g["step"])
    ctx.set_contacts(keys0)
    miss = ctx.count_missing()
    o = oracle.Oracle(s)
    ref = o.count_missing(_orc_state_from_gpu(s, g), keys0, step=g["step"])
    assert miss == ref and miss > 0


def test_config0_side_by_side_statistics(dem):
    """Config 0 (1,000 spheres, every-step detection) on both sides: the
    trajectories are chaotic, so bulk statistics are compared."""
    s = W.config0()
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    o = oracle.Oracle(s)
    st = o.state()
    ke_g, ke_o = [], []
    step = 0
    acs = None
    for blk in range(4):
        ctx.step(500)
        st, acs, _, step = o.run(st, 500, mode="every", acs=acs, step=step)
        g = ctx.get_state()
        ke_g.append(0.5 * (s.own_mass * (g["V"].astype(np.float64) ** 2).sum(1)).sum())
        ke_o.append(0.5 * (s.own_mass * (st["V"] ** 2).sum(1)).sum())
        zg, zo = g["X"][:, 2].mean(), st["X"][:, 2].mean()
        assert abs(zg - zo) < 2e-4
    ke_g, ke_o = np.array(ke_g), np.array(ke_o)
    assert np.all(np.abs(ke_g - ke_o) <= 0.05 * ke_o + 1e-9)


def test_fixed_schedule_tracks_the_oracle_fixed_schedule(dem):
    """The delayed fixed-margin schedule (k = 10, adoption 5 steps later,
    judged) on the GPU against the oracle's own run of the same schedule:
    the same number of detections and swaps, no missed contact on either
    side, the same final active set, and positions that agree to the level
    of the FP32 force law accumulated over the run."""
    import torch
    s = W.small_spheres(5, n=512, vel=0.3)
    steps = 300
    ctx = dem.DemContext(s, mode="fixed", k=10, lam=5, judge=True)
    ctx.set_state()
    st_g = ctx.step(steps, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
    g = ctx.get_state()
    keys, _ = ctx.get_contacts()
    o = oracle.Oracle(s)
    st, acs, st_o, _ = o.run(o.state(), steps, mode="fixed", k=10, lam=5, judge=True)
    assert st_g["misses"] == 0 and st_o["misses"] == 0
    assert st_g["cds"] == st_o["cds"] and st_g["swaps"] == st_o["swaps"]
    np.testing.assert_array_equal(keys, acs[0])
    assert np.sum(o.forces(st, acs[0], acs[1])["touch"]) > 0
    err = np.abs(g["X"] - st["X"]).max()
    print(f"max position difference after {steps} steps {err:.2e} m", flush=True)
    assert err <= 1e-7


def test_delayed_detection_stream_changes_nothing(dem):
    """The result does not depend on when the detection stream runs: the
    same fixed-margin run on two streams, once as is and once with a long
    queue of device copies enqueued on the detection stream ahead of it
    (every detection then finishes late and the dynamics stream waits at
    each adoption step), ends in the same state and set bit for bit, and
    equals every-step detection."""
    import torch
    s = W.small_clumps(9, n=300, vel=0.3, with_cylinder=True, spacing=0.0085)
    outs = []
    for delay in (False, True):
        c = dem.DemContext(s, mode="fixed", k=6, lam=3)
        c.set_state()
        dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
        if delay:
            a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            with torch.cuda.stream(kin):
                for _ in range(40):
                    b.copy_(a)
        st = c.step(60, dyn=dyn, kin=kin)
        torch.cuda.synchronize()
        outs.append((c.get_state(), c.get_contacts()[0], st))
        c.close()
    e = dem.DemContext(s, mode="every")
    e.set_state()
    e.step(60)
    ge = e.get_state()
    (g0, k0, s0), (g1, k1, s1) = outs
    assert s0["cds"] == s1["cds"] > 5
    np.testing.assert_array_equal(k0, k1)
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(g0[k], g1[k])
        np.testing.assert_array_equal(g0[k], ge[k])


def test_long_run_bulk_statistics(dem):
    """Config 0 run long enough to settle (20,000 every-step steps, 0.2 s:
    the spheres fall onto the floor) on both sides.  The trajectories are
    chaotic, so the packing fraction of the bottom 3 cm slab and the
    kinetic energy are compared every 2000 steps, against an interval set
    by the oracle itself: the spread between the oracle and the oracle
    started from the same state with one sphere moved by 2^-36 m (a
    rounding-level change); the GPU must stay within three times that
    spread plus 0.01 in packing fraction and 2 % of the kinetic energy."""
    s = W.config0()
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    o = oracle.Oracle(s)
    st_a = o.state()
    st_b = o.state()
    st_b["X"][0, 0] += 2.0 ** -36
    vol = 4.0 / 3.0 * np.pi * s.sph_rad ** 3
    lo, hi = np.asarray(s.domain_lo), np.asarray(s.domain_hi)
    slab = (hi[0] - lo[0]) * (hi[1] - lo[1]) * 0.03

    def stats(X, V):
        phi = vol[X[:, 2] < lo[2] + 0.03].sum() / slab
        ke = 0.5 * (s.own_mass * (np.asarray(V, dtype=np.float64) ** 2).sum(1)).sum()
        return phi, ke

    acs_a = acs_b = None
    step_a = step_b = 0
    rows = []
    for blk in range(10):
        ctx.step(2000)
        st_a, acs_a, _, step_a = o.run(st_a, 2000, mode="every", acs=acs_a, step=step_a)
        st_b, acs_b, _, step_b = o.run(st_b, 2000, mode="every", acs=acs_b, step=step_b)
        g = ctx.get_state()
        rows.append((stats(g["X"], g["V"]), stats(st_a["X"], st_a["V"]), stats(st_b["X"], st_b["V"])))
    ke0 = stats(s.X, s.V)[1]
    for (pg, kg), (pa, ka), (pb, kb) in rows:
        print(f"phi gpu {pg:.4f} oracle {pa:.4f} perturbed {pb:.4f}; KE gpu {kg:.4e} oracle {ka:.4e} "
              f"perturbed {kb:.4e}", flush=True)
        assert abs(pg - pa) <= 3 * abs(pb - pa) + 0.01
        assert abs(kg - ka) <= 3 * abs(kb - ka) + 0.02 * ka + 1e-3 * ke0
    # the bed has settled: most of the spheres' volume is in the bottom slab
    assert rows[-1][1][0] > 0.3
