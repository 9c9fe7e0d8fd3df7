"""Pins of the oracle's family tags (Sec. 2.2.2) and of the active-box
scheme built on them (Sec. 6.4).

* switched-off family pairs: binned == brute-force detection (two code
  paths), and the set is the unmasked set minus exactly the pairs whose
  families are switched off (spheres, walls and facets);
* fixed families: their owners' state never changes, the others move;
* a sphere resting on a fixed sphere settles at the static Hertz overlap of
  its weight with R = r/2 (closed form);
* active box: no dormant-dormant pair is listed, active-dormant pairs are.
"""
import numpy as np

import oracle
import workloads as W


def _fam_pairs(s, keys):
    i = (keys >> np.uint64(32)).astype(np.int64)
    j = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    fa = s.owner_family[s.sph_owner[i]].astype(np.int64)
    fb = np.zeros_like(fa)
    sph = j < s.n_spheres
    wal = (j >= s.n_spheres) & (j < s.n_spheres + s.n_walls)
    fac = j >= s.n_spheres + s.n_walls
    fb[sph] = s.owner_family[s.sph_owner[j[sph]]]
    fb[wal] = s.wall_family[j[wal] - s.n_spheres]
    fb[fac] = s.mesh_family[s.tri_mesh[j[fac] - s.n_spheres - s.n_walls]]
    return fa, fb


def test_switched_off_pairs_are_filtered_exactly():
    rng = np.random.default_rng(0)
    base = W.small_mixer_bed(3, n=300)
    # spheres pushed towards the blades so facets take part
    s = W.small_mixer_bed(3, n=300)
    fw = oracle.Oracle(s).facet_positions(0).reshape(-1, 3, 3)
    f = rng.integers(0, fw.shape[0], 120)
    s.X = s.X.copy()
    s.X[:120] = W.snap_pos(fw[f].mean(1) + rng.normal(0, 0.002, size=(120, 3)))
    base.X = s.X.copy()
    fam = rng.integers(0, 4, size=s.n_owners)
    W.set_families(s, fam, pair_off=[(0, 1), (2, 2), (3, 5), (1, 7)], wall_family=np.full(s.n_walls, 5),
                   mesh_family=np.array([7]))
    W.set_families(base, fam, wall_family=np.full(s.n_walls, 5), mesh_family=np.array([7]))
    m = 0.003
    o, ob = oracle.Oracle(s), oracle.Oracle(base)
    st = o.state()
    got = o.detect(st, m)
    np.testing.assert_array_equal(got, o.detect(st, m, brute=True))
    allk = ob.detect(ob.state(), m)
    fa, fb = _fam_pairs(base, allk)
    off = s.fam_pair_off.reshape(256, 256)[fa, fb] > 0
    assert off.sum() > 100 and (~off).sum() > 100
    np.testing.assert_array_equal(got, allk[~off])
    # every kind of partner is filtered: spheres, walls (family 5 with 3), facets (7 with 1)
    j = (allk & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert np.any(off & (j >= s.n_spheres + s.n_walls)) and np.any(off & (j >= s.n_spheres) & (j < s.n_spheres + s.n_walls))


def test_fixed_families_keep_their_state():
    s = W.small_spheres(7, n=343, vel=0.3)
    fam = (np.arange(s.n_owners) % 3 == 0).astype(np.uint8)
    W.set_families(s, fam, fixed=[1])
    o = oracle.Oracle(s)
    st0 = o.state()
    st, acs, stats, _ = o.run(o.state(), 300, mode="fixed", k=10, lam=5)
    fx = fam == 1
    for k in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(st[k][fx], st0[k][fx])
    assert np.all(np.linalg.norm(st["X"][~fx] - st0["X"][~fx], axis=1) > 0)
    # the fixed owners do take part in contacts
    i = (acs[0] >> np.uint64(32)).astype(np.int64)
    j = (acs[0] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    sph = j < s.n_spheres
    assert np.any(fx[s.sph_owner[i]] | (sph & fx[s.sph_owner[np.minimum(j, s.n_spheres - 1)]]))


def test_sphere_resting_on_a_fixed_sphere_settles_at_the_static_hertz_overlap():
    r = 0.005
    X = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2 * r - 2e-6]])
    s = W.assemble(np.full(2, -1), X, W._qid(2), np.zeros((2, 3)), np.zeros((2, 3)), [], r, None,
                   W.concat_walls(), W.materials(cor=0.05), (0, 0, -9.81), 2e-6, 0.0, -0.02 * np.ones(3),
                   0.03 * np.ones(3))
    W.set_families(s, np.array([1, 0]), fixed=[1])
    o = oracle.Oracle(s)
    st, acs, _, _ = o.run(o.state(), 40000, mode="every")
    rr = float(s.sph_rad[0])
    Es = 1.0 / (2 * (1 - 0.09) / float(s.mat_E[0]))
    m = float(s.own_mass[1])
    delta = (m * 9.81 / (4.0 / 3.0 * Es * np.sqrt(rr / 2))) ** (2.0 / 3.0)
    got = 2 * rr - (st["X"][1, 2] - st["X"][0, 2])
    assert abs(got - delta) <= 1e-3 * delta, (got, delta)
    assert abs(st["V"][1, 2]) < 1e-5
    np.testing.assert_array_equal(st["X"][0], X[0])


def test_active_box_lists_no_dormant_pair():
    s = W.small_spheres(8, n=512, vel=0.2)
    c = s.X.mean(0)
    W.active_box(s, c - 0.01, c + 0.01)
    o = oracle.Oracle(s)
    keys = o.detect(o.state(), 0.002)
    fa, fb = _fam_pairs(s, keys)
    assert not np.any((fa == 1) & (fb == 1))
    assert np.any((fa == 0) & (fb == 0)) and np.any(fa != fb)
    assert 0 < (s.owner_family == 0).sum() < s.n_owners // 2
