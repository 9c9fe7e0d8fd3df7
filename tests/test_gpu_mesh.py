"""Parity of the sphere-facet path of the HIP library (rigid triangle meshes
with prescribed motion, Sec. 2.4; the bladed mixer of Sec. 5) with the FP64
oracle, through the C ABI.

Bars as for spheres and walls: contact sets bit-exact (both sides evaluate
|x - closest point|^2 < (r + 2m)^2 in FP64 on the same facet vertices, the
mesh pose being computed on the host on both sides); forces, history and
one-step increments within 1e-5 relative; delayed detection equal to
every-step detection bit for bit.
"""
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


def near_facets(seed, n=600, step=0, off=(0.3, 1.0), margin=0.0002):
    """Spheres around the impeller of the small mixer at the pose of `step`:
    random points of random facets pushed off the facet plane (either side)
    by U(off) r plus up to 3 m, and a fifth placed around a facet vertex, so
    face, edge and vertex regions all occur."""
    s = W.small_mixer_bed(seed, n=n)
    s.margin = margin
    fw = oracle.Oracle(s).facet_positions(step).reshape(-1, 3, 3)
    rng = np.random.default_rng(seed)
    f = rng.integers(0, fw.shape[0], n)
    u, v = rng.uniform(size=(2, n))
    flip = u + v > 1.0
    u[flip], v[flip] = 1.0 - u[flip], 1.0 - v[flip]
    a, b, c = fw[f, 0], fw[f, 1], fw[f, 2]
    p = a + u[:, None] * (b - a) + v[:, None] * (c - a)
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    r = s.sph_rad
    d = rng.uniform(*off, size=n) * r + rng.uniform(0.0, 3.0 * margin, size=n)
    X = p + (rng.choice([-1.0, 1.0], size=n) * d)[:, None] * nrm
    vert = rng.random(n) < 0.2
    dirv = rng.normal(size=(n, 3))
    dirv /= np.linalg.norm(dirv, axis=1, keepdims=True)
    X[vert] = a[vert] + dirv[vert] * (rng.uniform(*off, size=vert.sum()) * r[vert])[:, None]
    s.X = W.snap_pos(X)
    return s


def _keys_split(s, keys):
    j = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    return j >= s.n_spheres + s.n_walls


@pytest.mark.parametrize("step", [0, 7777])
@pytest.mark.parametrize("margin_scale", [0.0, 1.0])
def test_mesh_contact_sets_bit_exact(dem, step, margin_scale):
    s = near_facets(1, step=step)
    m = margin_scale * s.margin
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=48 * s.n_spheres)
    ctx.set_state(step=step)
    n = ctx.detect_contacts(m)
    keys, hist = ctx.get_contacts()
    assert n == keys.size
    o = oracle.Oracle(s)
    ref = o.detect(o.state(), m, step=step)
    print(f"step {step} m {m}: contacts {keys.size} facet {_keys_split(s, ref).sum()}")
    assert _keys_split(s, ref).sum() > 100
    np.testing.assert_array_equal(keys, ref)


def fine_floor(n_cells=24, cell=0.0005, r=0.003):
    """One sphere pressed 0.3 mm into a finely meshed floor: its row holds
    far more facets than the 16 staged partners of the detection."""
    s = W.assemble(np.full(2, -1), np.array([[0.0, 0.0, r - 3e-4], [0.02, 0.02, 0.02]]), W._qid(2),
                   np.zeros((2, 3)), np.zeros((2, 3)), [], r, None, W.concat_walls(), W.materials(),
                   (0, 0, -9.81), 1e-6, 0.0004, -0.03 * np.ones(3), 0.03 * np.ones(3), name="fine_floor")
    L = n_cells * cell
    tri = W.quad_grid((-0.5 * L, -0.5 * L, 0.0), (L, 0, 0), (0, L, 0), n_cells, n_cells)
    return W.add_meshes(s, dict(tri=tri, origin=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 3.0)))


@pytest.mark.parametrize("m", [0.0, 0.0004])
def test_mesh_rows_longer_than_the_stage_bit_exact(dem, m):
    s = fine_floor()
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=1024)
    ctx.set_state(step=11)
    ctx.detect_contacts(m)
    keys, _ = ctx.get_contacts()
    o = oracle.Oracle(s)
    ref = o.detect(o.state(), m, step=11)
    assert (ref >> np.uint64(32) == 0).sum() > 16
    np.testing.assert_array_equal(keys, ref)


def test_mesh_without_facets_changes_nothing(dem):
    """A mesh with no facets: the same contact set and trajectory as no mesh."""
    s = W.small_spheres(4, n=216, vel=0.3)
    e = W.small_spheres(4, n=216, vel=0.3)
    W.add_meshes(e, dict(tri=np.zeros((0, 3, 3)), omega=(0.0, 0.0, 1.0)))
    assert e.n_mesh == 1 and e.n_tri == 0
    out = []
    for sysm in (s, e):
        c = dem.DemContext(sysm, mode="fixed", k=6, lam=3)
        c.set_state()
        c.step(60)
        out.append((c.get_state(), c.get_contacts()[0]))
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(out[0][0][k], out[1][0][k])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_mesh_forces_match_oracle(dem):
    s = near_facets(2, step=4321, off=(0.85, 1.0))
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=48 * s.n_spheres)
    ctx.set_state(step=4321)
    ctx.detect_contacts(s.margin)
    keys, _ = ctx.get_contacts()
    rng = np.random.default_rng(5)
    hist = W.f32(rng.normal(0.0, 3e-6, size=(keys.size, 4))).astype(np.float32)
    hist[:, 3] = 0.0
    ctx.set_contacts(keys, hist)
    ctx.forces()
    Fo, To, Fc = ctx.get_forces(keys.size)
    _, h2 = ctx.get_contacts()
    g = ctx.get_state()
    o = oracle.Oracle(s)
    ost = {"X": g["X"].copy(), "q": g["q"].copy(), "V": g["V"].astype(np.float64), "W": g["W"].astype(np.float64)}
    ref = o.forces(ost, keys, hist.astype(np.float64), step=g["step"])
    touch = ref["touch"] > 0
    fac = _keys_split(s, keys)
    assert (touch & fac).sum() > 50
    Fn = np.linalg.norm(ref["Fc"], axis=1)
    Fmed = np.median(Fn[touch])
    rel = np.linalg.norm(Fc - ref["Fc"], axis=1) / np.maximum(Fn, 1e-3 * Fmed)
    print(f"contacts {keys.size} facet {fac.sum()} touching facet {(touch & fac).sum()} max rel {rel.max():.2e}")
    assert rel.max() <= 1e-5
    assert np.all(Fc[~touch] == 0.0) and np.all(h2[~touch] == 0.0)
    hn = np.linalg.norm(ref["hist"][:, :3], axis=1)
    herr = np.linalg.norm(h2[:, :3] - ref["hist"][:, :3], axis=1) / np.maximum(hn, 1e-3 * np.median(hn[touch]))
    assert herr.max() <= 1e-5
    L1 = np.zeros(s.n_owners)
    ks = (keys >> np.uint64(32)).astype(np.int64)
    js = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.add.at(L1, s.sph_owner[ks], Fn)
    sph = js < s.n_spheres
    np.add.at(L1, s.sph_owner[js[sph]], Fn[sph])
    assert np.all(np.linalg.norm(Fo - ref["Fo"], axis=1) <= 1e-5 * np.maximum(L1, 1e-3 * Fmed) + 1e-30)
    assert np.all(np.linalg.norm(To - ref["To"], axis=1) <= 1e-5 * np.maximum(L1 * 0.006, 3e-6 * Fmed) + 1e-30)


def test_mesh_one_step_matches_oracle(dem):
    s = near_facets(3, step=100, off=(0.9, 1.0))
    ctx = dem.DemContext(s, mode="every", capacity=48 * s.n_spheres)
    ctx.set_state(step=100)
    g0 = ctx.get_state()
    before = {"X": g0["X"].copy(), "q": g0["q"].copy(), "V": g0["V"].astype(np.float64),
              "W": g0["W"].astype(np.float64)}
    ctx.step(1)
    g1 = ctx.get_state()
    o = oracle.Oracle(s)
    st1, acs, _, _ = o.run({k: v.copy() for k, v in before.items()}, 1, mode="every", step=100)
    keys = acs[0]
    assert _keys_split(s, keys).sum() > 50
    out = o.forces(before, keys, np.zeros((keys.size, 3)), step=100)
    Fn = np.linalg.norm(out["Fc"], axis=1)
    L1 = np.zeros(s.n_owners)
    ks = (keys >> np.uint64(32)).astype(np.int64)
    js = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    np.add.at(L1, s.sph_owner[ks], Fn)
    sph = js < s.n_spheres
    np.add.at(L1, s.sph_owner[js[sph]], Fn[sph])
    h = s.dt
    dv_g = g1["V"].astype(np.float64) - before["V"]
    dv_o = st1["V"] - before["V"]
    tol_v = 1e-5 * np.linalg.norm(dv_o, axis=1) + np.spacing(np.abs(g1["V"]).max(1).astype(np.float32)) \
        + 1e-5 * h * L1 / s.own_mass
    assert np.all(np.linalg.norm(dv_g - dv_o, axis=1) <= tol_v)
    dx_g, dx_o = g1["X"] - before["X"], st1["X"] - before["X"]
    tol_x = 1e-5 * np.linalg.norm(dx_o, axis=1) + h * np.linalg.norm(dv_g - dv_o, axis=1) + 2.0 ** -37
    assert np.all(np.linalg.norm(dx_g - dx_o, axis=1) <= tol_x)
    dw_g = g1["W"].astype(np.float64) - before["W"]
    dw_o = st1["W"] - before["W"]
    tol_w = 1e-5 * np.linalg.norm(dw_o, axis=1) + 4 * np.spacing(np.abs(g1["W"]).max(1).astype(np.float32)) \
        + 1e-5 * h * L1 * 0.01 / s.own_moi.min(1)
    assert np.all(np.linalg.norm(dw_g - dw_o, axis=1) <= tol_w)


def _run(dem, s, n, **kw):
    import torch
    two = kw.pop("two_streams", False)
    c = dem.DemContext(s, **kw)
    c.set_state()
    st = c.step(n, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream()) if two else c.step(n)
    g = c.get_state()
    keys, hist = c.get_contacts()
    c.close()
    return st, g, keys, hist


def test_mixer_delayed_and_adaptive_equal_every_step_bitwise(dem):
    """The blades sweep the small bed: facet contacts emerge and vanish.
    Delayed detection (fixed interval, two streams) and the adaptive policy
    (its margin covers the fastest mesh point) reproduce every-step
    detection bit for bit, with no contact missed."""
    s = W.small_mixer_bed(5, n=500)
    n = 800
    _, ga, ka, _ = _run(dem, s, n, mode="every")
    seen = _keys_split(s, ka).sum()
    st_f, gb, _, _ = _run(dem, s, n, mode="fixed", k=10, lam=5, judge=True, two_streams=True)
    st_a, gc, _, _ = _run(dem, s, n, mode="adaptive", k=10, lam=2, k_max=8, judge=True, two_streams=True)
    print(f"facet contacts at the end {seen}; fixed cds {st_f['cds']} adaptive cds {st_a['cds']}")
    assert seen > 5
    assert st_f["misses"] == 0 and st_a["misses"] == 0
    for g in (gb, gc):
        for k in ("X", "V", "W"):
            np.testing.assert_array_equal(ga[k], g[k])


def test_mixer_fused_equals_two_kernel_path_bitwise(dem):
    s = W.small_mixer_bed(6, n=500)
    out = [_run(dem, s, 800, mode="fixed", k=6, lam=3, dyn_path=p, two_streams=True) for p in (0, 1)]
    (_, ga, ka, ha), (_, gb, kb, hb) = out
    assert _keys_split(s, ka).sum() > 0
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])
    np.testing.assert_array_equal(ka, kb)
    np.testing.assert_array_equal(ha, hb)


def test_mixer_trajectory_tracks_oracle(dem):
    """800 every-step steps of the swept bed on both sides (the blades hit
    spheres at up to 3 m/s): positions agree to the level of the FP32 force
    law accumulated over the run."""
    s = W.small_mixer_bed(7, n=300)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    g0 = ctx.get_state()
    st = {"X": g0["X"].copy(), "q": g0["q"].copy(), "V": g0["V"].astype(np.float64),
          "W": g0["W"].astype(np.float64)}
    o = oracle.Oracle(s)
    ctx.step(800)
    g = ctx.get_state()
    st1, acs, _, _ = o.run(st, 800, mode="every")
    keys, _ = ctx.get_contacts()
    assert _keys_split(s, acs[0]).sum() > 0 and _keys_split(s, keys).sum() > 0
    err = np.abs(g["X"] - st1["X"]).max()
    print(f"max position difference after 800 steps {err:.2e} m")
    assert err <= 1e-7


def test_mesh_judge_counts_missing_like_oracle(dem):
    """A set detected at one step judged at a later pose of the impeller:
    the facet contacts that appeared meanwhile are counted as the oracle
    counts them."""
    s = near_facets(8, step=0, off=(0.9, 1.3))
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=48 * s.n_spheres)
    ctx.set_state(step=0)
    ctx.detect_contacts(0.0)
    keys, _ = ctx.get_contacts()
    g = ctx.get_state()
    later = 400   # the impeller turns 0.0126 rad meanwhile: up to 0.6 mm at the tips
    ctx.set_state(X=g["X"], q=g["q"], V=g["V"], W=g["W"], step=later)
    ctx.set_contacts(keys)
    miss = ctx.count_missing()
    o = oracle.Oracle(s)
    ref = o.count_missing(o.state(), keys, step=later)
    print(f"set {keys.size} missing {miss} oracle {ref}")
    assert ref > 0
    assert miss == ref


def clumps_on_mesh_floor(seed=2, n=150):
    """Tri- and five-sphere clumps and single spheres thrown down at 2 m/s
    onto a facet floor 0.3 mm below the lowest sphere, the floor spinning at
    5 rad/s about z (friction drags the clumps round)."""
    s = W.small_clumps(seed, n=n, vel=0.3)
    s.V[:, 2] = -2.0
    o = oracle.Oracle(s)
    xs = o.sphere_centres(o.state())
    zf = float((xs[:, 2] - s.sph_rad).min()) - 0.0003
    L = float(s.domain_hi[0] - s.domain_lo[0]) - 0.004
    tri = W.quad_grid((-0.5 * L, -0.5 * L, 0.0), (L, 0, 0), (0, L, 0), 8, 8)
    return W.add_meshes(s, dict(tri=tri, origin=(0.0, 0.0, zf), omega=(0.0, 0.0, 5.0)))


def test_clumps_on_a_mesh_floor(dem):
    """Clump systems with facets: delayed detection on two streams equals
    every-step detection bit for bit; after the run the contact set equals
    the oracle's and the forces agree within 1e-5."""
    s = clumps_on_mesh_floor()
    _, ga, ka, _ = _run(dem, s, 300, mode="every")
    st_f, gb, _, _ = _run(dem, s, 300, mode="fixed", k=6, lam=3, judge=True, two_streams=True)
    assert st_f["misses"] == 0
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=64 * s.n_spheres)
    ctx.set_state(X=ga["X"], q=ga["q"], V=ga["V"], W=ga["W"], step=ga["step"])
    ctx.detect_contacts(s.margin)
    keys, _ = ctx.get_contacts()
    g = ctx.get_state()
    st = {"X": g["X"].copy(), "q": g["q"].copy(), "V": g["V"].astype(np.float64), "W": g["W"].astype(np.float64)}
    o = oracle.Oracle(s)
    np.testing.assert_array_equal(keys, o.detect(st, s.margin, step=g["step"]))
    fac = _keys_split(s, keys)
    ctx.forces()
    _, _, Fc = ctx.get_forces(keys.size)
    ref = o.forces(st, keys, np.zeros((keys.size, 4)), step=g["step"])
    touch = ref["touch"] > 0
    print(f"contacts {keys.size} facet {fac.sum()} touching facet {(touch & fac).sum()}")
    assert (touch & fac).sum() > 5
    Fn = np.linalg.norm(ref["Fc"], axis=1)
    rel = np.linalg.norm(Fc - ref["Fc"], axis=1) / np.maximum(Fn, 1e-3 * np.median(Fn[touch]))
    assert rel.max() <= 1e-5
