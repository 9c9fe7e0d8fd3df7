"""Edge cases of the HIP path against the oracle: empty and tiny inputs,
predicate boundaries (exact equality is not a contact), ragged sizes around
the kernels' block and tile sizes."""
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


def _spheres(X, r, V=None, walls=None, margin=0.0, lo=-1.0, hi=1.0):
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    V = np.zeros((n, 3)) if V is None else np.asarray(V, dtype=np.float64)
    return W.assemble(np.full(n, -1), X, W._qid(n), V, np.zeros((n, 3)), [], r, None,
                      walls if walls is not None else W.concat_walls(), W.materials(), (0, 0, -9.81), 1e-5, margin,
                      lo * np.ones(3), hi * np.ones(3))


def test_single_sphere_free_fall(dem):
    s = _spheres([[0.0, 0.0, 0.5]], 0.01)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    assert ctx.detect_contacts(0.0) == 0
    ctx.step(100)
    g = ctx.get_state()
    o = oracle.Oracle(s)
    st, *_ = o.run(o.state(), 100, mode="every")
    np.testing.assert_allclose(g["V"], st["V"], rtol=1e-6)
    np.testing.assert_allclose(g["X"], st["X"], rtol=0, atol=1e-9)


def test_no_contacts_anywhere(dem):
    X = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(5), indexing="ij"), -1).reshape(-1, 3) * 0.05
    s = _spheres(X - 0.1, 0.005, margin=0.0005)
    ctx = dem.DemContext(s, mode="fixed", k=10, lam=3)
    ctx.set_state()
    stats = ctx.step(50)
    assert stats["n_contacts"] == 0
    keys, hist = ctx.get_contacts()
    assert keys.size == 0


def test_exact_touch_is_not_a_contact(dem):
    """Centres 0.5 m apart with radii 0.25 m (all exact in binary): the gap is
    exactly zero, which the strict predicate does not count."""
    s = _spheres([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.0, 0.499755859375]], 0.25, lo=-1.0, hi=1.5)
    s.gravity[:] = 0.0
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    ctx.detect_contacts(0.0)
    keys, _ = ctx.get_contacts()
    o = oracle.Oracle(s)
    ref = o.detect(o.state(), 0.0)
    np.testing.assert_array_equal(keys, ref)
    assert keys.tolist() == [2]   # only the pair (0, 2) overlaps


def test_exact_wall_touch_is_not_a_contact(dem):
    walls = W.concat_walls(W.plane((0, 0, 0), (0, 0, 1)), W.plane((0, 0, 0.75), (0, 0, -1)))
    s = _spheres([[0.0, 0.0, 0.25], [0.6, 0.0, 0.5]], 0.25, walls=walls, lo=-1.0, hi=1.5)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    ctx.detect_contacts(0.0)
    keys, _ = ctx.get_contacts()
    assert keys.size == 0
    o = oracle.Oracle(s)
    np.testing.assert_array_equal(keys, o.detect(o.state(), 0.0))


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097])
def test_ragged_sizes_detection_and_step(dem, n):
    s = W.small_spheres(n, n=n, vel=0.3)
    ctx = dem.DemContext(s, mode="fixed", k=5, lam=2)
    ctx.set_state()
    m = s.margin
    ctx.detect_contacts(m)
    keys, _ = ctx.get_contacts()
    o = oracle.Oracle(s)
    np.testing.assert_array_equal(keys, o.detect(o.state(), m))
    a = dem.DemContext(s, mode="every")
    a.set_state()
    a.step(20)
    ctx.set_state()
    ctx.step(20)
    ga, gb = a.get_state(), ctx.get_state()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(ga[k], gb[k])


def test_clump_overlapping_own_spheres_excluded(dem):
    s = W.small_clumps(3, n=8, with_singles=False, spacing=0.02)
    o = oracle.Oracle(s)
    ctx = dem.DemContext(s, mode="every")
    ctx.set_state()
    ctx.detect_contacts(0.0)
    keys, _ = ctx.get_contacts()
    np.testing.assert_array_equal(keys, o.detect(o.state(), 0.0))
    i = (keys >> np.uint64(32)).astype(np.int64)
    j = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    sph = j < s.n_spheres
    assert np.all(s.sph_owner[i[sph]] != s.sph_owner[j[sph]])
