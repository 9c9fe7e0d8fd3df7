"""Family tags (Sec. 2.2.2) and the active-box scheme (Sec. 6.4) on the GPU,
through the C ABI, against the FP64 oracle and against the library's own
schedules:

* switched-off family pairs: contact sets bit-exact with the oracle
  (spheres, walls, facets; margin 0 and m) and the judge's count equal;
* fixed families: their owners' state bitwise unchanged over a run; one step
  against the oracle; delayed == every-step detection and the fused step ==
  the two-kernel form, bit for bit, for spheres and clumps;
* a moving active box: the set rebuilt at the move equals the oracle's under
  the new tags, newly dormant owners keep their state from the move on, and
  the delayed run equals the every-step run bit for bit through the move.
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


def tagged_mixer(seed=3, n=300):
    """The small mixer bed with a third of its spheres pushed onto the blades,
    four owner families, the walls in family 5, the impeller in family 7, and
    the pairs (0,1), (2,2), (3,5), (1,7) switched off."""
    rng = np.random.default_rng(seed)
    s = W.small_mixer_bed(seed, n=n)
    fw = oracle.Oracle(s).facet_positions(0).reshape(-1, 3, 3)
    k = n // 3
    f = rng.integers(0, fw.shape[0], k)
    s.X = s.X.copy()
    s.X[:k] = W.snap_pos(fw[f].mean(1) + rng.normal(0, 0.002, size=(k, 3)))
    fam = rng.integers(0, 4, size=s.n_owners)
    return W.set_families(s, fam, pair_off=[(0, 1), (2, 2), (3, 5), (1, 7)],
                          wall_family=np.full(s.n_walls, 5), mesh_family=np.array([7]))


def _gstate(g):
    return {"X": g["X"].copy(), "q": g["q"].copy(), "V": g["V"].astype(np.float64), "W": g["W"].astype(np.float64)}


@pytest.mark.parametrize("m", [0.0, 0.003])
def test_switched_off_pairs_bit_exact(dem, m):
    s = tagged_mixer()
    ctx = dem.DemContext(s, mode="fixed", margin=0.003, capacity=64 * s.n_spheres)
    ctx.set_state()
    ctx.detect_contacts(m)
    keys, _ = ctx.get_contacts()
    o = oracle.Oracle(s)
    ref = o.detect(o.state(), m)
    print(f"m {m}: {keys.size} contacts")
    assert ref.size > 100
    np.testing.assert_array_equal(keys, ref)


def test_judge_counts_switched_off_pairs_like_oracle(dem):
    s = tagged_mixer(4)
    ctx = dem.DemContext(s, mode="fixed", margin=0.003, capacity=64 * s.n_spheres)
    ctx.set_state()
    ctx.detect_contacts(0.0)
    keys, _ = ctx.get_contacts()
    rng = np.random.default_rng(1)
    sub = np.sort(keys[rng.random(keys.size) < 0.7])
    ctx.set_contacts(sub)
    miss = ctx.count_missing()
    o = oracle.Oracle(s)
    ref = o.count_missing(o.state(), sub)
    assert ref > 10 and miss == ref


def fixed_spheres(seed=7, n=512, dormant=False):
    """Every third owner fixed; `dormant`: also switched off with the walls
    (family 2), so the fixed spheres leave the binning (dormant index)."""
    s = W.small_spheres(seed, n=n, vel=0.3)
    fam = (np.arange(s.n_owners) % 3 == 0).astype(np.uint8)
    if dormant:
        return W.set_families(s, fam, pair_off=[(1, 1), (1, 2)], fixed=[1], wall_family=np.full(s.n_walls, 2))
    return W.set_families(s, fam, pair_off=[(1, 1)], fixed=[1])


def fixed_clumps(seed=6, n=300, dormant=False):
    s = W.small_clumps(seed, n=n, vel=0.3, spacing=0.0080)
    fam = (np.arange(s.n_owners) % 4 == 1).astype(np.uint8)
    if dormant:
        return W.set_families(s, fam, pair_off=[(1, 1), (1, 2)], fixed=[1], wall_family=np.full(s.n_walls, 2))
    return W.set_families(s, fam, pair_off=[(1, 1)], fixed=[1])


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


@pytest.mark.parametrize("name", ["spheres", "clumps", "spheres_dormant", "clumps_dormant"])
def test_fixed_families_schedules_bitwise(dem, name):
    dorm = name.endswith("dormant")
    s = fixed_spheres(dormant=dorm) if name.startswith("spheres") else fixed_clumps(dormant=dorm)
    fx = s.fam_fixed[s.owner_family] > 0
    _, ga, ka, ha = _run(dem, s, 300, mode="every")
    st_f, gb, _, _ = _run(dem, s, 300, mode="fixed", k=10, lam=5, judge=True, two_streams=True)
    _, gc, kc, hc = _run(dem, s, 300, mode="fixed", k=10, lam=5, dyn_path=1, two_streams=True)
    _, gd, kd, hd = _run(dem, s, 300, mode="fixed", k=10, lam=5, dyn_path=0, two_streams=True)
    # (free owners bouncing off fixed ones can outrun the margin: the judge
    # then repairs the set, and the run still equals every-step detection)
    print(f"{name}: judged misses {st_f['misses']}, repairs {st_f['repairs']}")
    for k in ("X", "V", "W", "q"):
        np.testing.assert_array_equal(ga[k], gb[k])
        np.testing.assert_array_equal(gc[k], gd[k])
    np.testing.assert_array_equal(kc, kd)
    np.testing.assert_array_equal(hc, hd)
    # fixed owners: unchanged (velocities zero), the others moved
    np.testing.assert_array_equal(ga["X"][fx], s.X[fx])
    assert np.all(ga["V"][fx] == 0) and np.all(ga["W"][fx] == 0)
    assert np.all(np.any(ga["X"][~fx] != s.X[~fx], axis=1))
    # fixed owners take part in contacts with the free ones
    i = (ka >> np.uint64(32)).astype(np.int64)
    j = (ka & np.uint64(0xFFFFFFFF)).astype(np.int64)
    sph = j < s.n_spheres
    fi = fx[s.sph_owner[i]]
    fj = fx[s.sph_owner[np.where(sph, j, 0)]] & sph
    assert np.any(fi != fj) and not np.any(fi & fj)


@pytest.mark.parametrize("dormant", [False, True])
@pytest.mark.parametrize("m", [0.0, 0.0002])
def test_fixed_contact_sets_bit_exact(dem, dormant, m):
    """With fixed families, and with dormant ones (left out of the binning,
    found through their static index), the sets equal the oracle's."""
    for s in (fixed_spheres(12, n=729, dormant=dormant), fixed_clumps(13, n=216, dormant=dormant)):
        ctx = dem.DemContext(s, mode="fixed", margin=0.0002, capacity=32 * s.n_spheres)
        ctx.set_state()
        ctx.detect_contacts(m)
        keys, _ = ctx.get_contacts()
        o = oracle.Oracle(s)
        ref = o.detect(o.state(), m)
        assert ref.size > 50
        np.testing.assert_array_equal(keys, ref)
        ctx.close()


def test_dormant_rows_longer_than_the_stage(dem):
    """A large active sphere covered by 60 small dormant ones: its row (60
    dormant partners) goes through the overflow path of the compaction,
    which finds dormant partners through the index too."""
    import test_gpu_parity as P
    s = P.cluster()
    fam = np.ones(s.n_owners, dtype=np.uint8)
    fam[0] = 0
    W.set_families(s, fam, pair_off=[(1, 1), (1, 2)], fixed=[1], wall_family=np.full(s.n_walls, 2))
    ctx = dem.DemContext(s, mode="fixed", margin=s.margin, capacity=64 * s.n_spheres)
    ctx.set_state()
    for m in (0.0, s.margin):
        ctx.detect_contacts(m)
        keys, _ = ctx.get_contacts()
        o = oracle.Oracle(s)
        ref = o.detect(o.state(), m)
        assert (ref >> np.uint64(32) == 0).sum() > 16
        np.testing.assert_array_equal(keys, ref)


def test_fixed_one_step_matches_oracle(dem):
    s = fixed_spheres(9)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    g0 = ctx.get_state()
    before = _gstate(g0)
    ctx.step(1)
    g1 = ctx.get_state()
    o = oracle.Oracle(s)
    st1, acs, _, _ = o.run({k: v.copy() for k, v in before.items()}, 1, mode="every")
    keys = acs[0]
    out = o.forces(before, keys, np.zeros((keys.size, 3)))
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
    fx = s.fam_fixed[s.owner_family] > 0
    np.testing.assert_array_equal(g1["X"][fx], before["X"][fx])


def test_moving_active_box(dem):
    """The active box moves after 150 steps (the paper updates its boxes
    as the rover advances)."""
    import torch
    s = W.small_spheres(11, n=729, vel=0.3)
    c = s.X.mean(0)
    box1 = (c - np.array([0.02, 0.03, 0.03]), c + np.array([0.005, 0.03, 0.03]))
    box2 = (c - np.array([0.005, 0.03, 0.03]), c + np.array([0.02, 0.03, 0.03]))
    W.active_box(s, *box1)
    s2 = W.small_spheres(11, n=729, vel=0.3)
    out = []
    for mode in ("every", "fixed"):
        ctx = dem.DemContext(s, mode=mode, k=8, lam=4, judge=mode == "fixed")
        ctx.set_state()
        dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
        ctx.step(150, dyn=dyn, kin=kin)
        g = ctx.get_state()
        inside = np.all((g["X"] >= box2[0]) & (g["X"] <= box2[1]), axis=1)
        fam2 = np.where(inside, 0, 1).astype(np.uint8)
        W.set_families(s2, fam2, pair_off=[(1, 1)], fixed=[1])
        ctx.set_families(s2.owner_family, None, None, s2.fam_pair_off, s2.fam_fixed)
        gm = ctx.get_state()
        keys, _ = ctx.get_contacts()
        if mode == "fixed":
            # the rebuilt set is the oracle's under the new tags
            o = oracle.Oracle(s2)
            np.testing.assert_array_equal(keys, o.detect(_gstate(gm), s.margin, step=gm["step"]))
        st = ctx.step(150, dyn=dyn, kin=kin)
        if mode == "fixed":
            assert st["misses"] == 0
        ge = ctx.get_state()
        dormant = fam2 == 1
        np.testing.assert_array_equal(ge["X"][dormant], gm["X"][dormant])
        assert np.all(ge["V"][dormant] == 0)
        was_active = np.all((s.X >= box1[0]) & (s.X <= box1[1]), axis=1)
        assert np.any(dormant & was_active) and np.any(~dormant & ~was_active)
        out.append(ge)
        ctx.close()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_set_families_rejects_an_asymmetric_table(dem):
    s = W.small_spheres(1, n=64)
    ctx = dem.DemContext(s, mode="fixed")
    off = np.zeros((256, 256), dtype=np.uint8)
    off[1, 2] = 1
    with pytest.raises(dem.DemError, match="symmetric"):
        ctx.set_families(np.zeros(s.n_owners, np.uint8), None, None, off.reshape(-1), None)
