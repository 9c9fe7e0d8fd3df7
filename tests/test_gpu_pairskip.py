"""Pair skipping: in the fused step (single-sphere systems, dense sets) and
in the split step of clump systems.

A pair whose key says it cannot touch is given exactly what evaluating it
would give (no force, zero history), so runs with skipping and runs that
evaluate every pair must end bit for bit in the same state, set and
history: over long chains (fixed and learned intervals), on a bed swept by
a turning mesh, against a moving cylinder and plane walls, and for clumps
whose spheres are carried towards each other mostly by their rotation.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dem():
    import os
    import paper_2311_04648_amd as d
    if not os.path.exists(d.LIB_PATH):
        from paper_2311_04648_amd import build
        build.build()
    d._torch()
    return d


def _run(dem, s, n, skip, **kw):
    import torch
    c = dem.DemContext(s, pair_skip=skip, **kw)
    c.set_state()
    st = c.step(n, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
    g = c.get_state()
    keys, hist = c.get_contacts()
    c.close()
    return st, g, keys, hist


def _same(a, b):
    for k in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(a[1][k], b[1][k])
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])


def cylinder_cloud(seed=3, n=600):
    """A packed sphere cloud in a box with a cylinder (radius 1 cm, axis
    along y) driven through it at 1 m/s: plane and cylinder walls, both
    the radial and the axial bound of the cylinder's gap."""
    rng = np.random.default_rng(seed)
    side = int(math.ceil(n ** (1 / 3)))
    sp = 0.0062
    base = W.lattice((side, side, side), sp, -0.5 * (side - 1) * sp * np.ones(3), n_take=n)
    rad = rng.uniform(0.0025, 0.003, size=n)
    X = base + rng.uniform(-0.0003, 0.0003, size=(n, 3))
    V = rng.normal(0.0, 0.05, size=(n, 3))
    half = 0.5 * side * sp + 0.02
    lo, hi = -half * np.ones(3), half * np.ones(3)
    cyl = W.cylinder((-half + 0.012, 0.0, 0.0), (0, 1, 0), 0.01, 0.5 * half, vel=(1.0, 0.0, 0.0))
    walls = W.concat_walls(W.box_walls(lo, hi), cyl)
    return W.assemble(np.full(n, -1), X, W._qid(n), V, np.zeros((n, 3)), [], rad, None, walls, W.materials(),
                      (0, 0, -9.81), 5e-6, 0.0006, lo, hi, name="cylinder_cloud")


@pytest.mark.parametrize("mode,k", [("fixed", 10), ("fixed", 60), ("learned", 10), ("every", 1)])
def test_mixer_bed_skipping_changes_nothing(dem, mode, k):
    s = W.small_mixer_bed(4, n=500)
    kw = dict(mode=mode, k=k, lam=5, dyn_path=2, k_max=200)
    a = _run(dem, s, 1200, True, **kw)
    b = _run(dem, s, 1200, False, **kw)
    print(f"{mode} k={k}: {a[2].size} pairs at the end, cds {a[0]['cds']}", flush=True)
    assert a[2].size > 0
    _same(a, b)


@pytest.mark.parametrize("mode", ["fixed", "learned"])
def test_moving_cylinder_and_walls_skipping_changes_nothing(dem, mode):
    s = cylinder_cloud()
    kw = dict(mode=mode, k=40, lam=5, dyn_path=2, k_max=200)
    a = _run(dem, s, 3000, True, **kw)
    b = _run(dem, s, 3000, False, **kw)
    ki = (a[2] >> np.uint64(32)).astype(np.int64)
    kj = (a[2] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    walls = np.unique(kj[kj >= s.n_spheres] - s.n_spheres)
    print(f"{mode}: {a[2].size} pairs, wall pairs with walls {walls.tolist()}, cds {a[0]['cds']}", flush=True)
    # the cylinder (the last wall) is in the set at the end
    assert s.n_walls - 1 in walls.tolist()
    _same(a, b)


def test_skipping_equals_the_two_kernel_form(dem):
    """The two-kernel form evaluates every pair every step."""
    s = W.small_mixer_bed(6, n=500)
    a = _run(dem, s, 800, True, mode="fixed", k=20, lam=5, dyn_path=0)
    b = _run(dem, s, 800, True, mode="fixed", k=20, lam=5, dyn_path=1)
    _same(a, b)


def _touching(st):
    return int(np.count_nonzero(np.any(st[3][:, :3] != 0.0, axis=1))) if st[3].size else 0


@pytest.mark.parametrize("mode,k", [("fixed", 10), ("fixed", 20), ("learned", 10), ("every", 1)])
def test_clump_split_step_skipping_changes_nothing(dem, mode, k):
    """Clumps, single spheres, a moving plane wall and a driven cylinder in
    the split step (the streaming kernel and the kernel over the owners
    with contacts).  (Fixed intervals of 40 steps and more miss contacts in
    this cloud and end diverged, with skipping or without.)"""
    s = W.small_clumps(5, n=343, spacing=0.0095, vel=0.2, with_cylinder=True)
    kw = dict(mode=mode, k=k, lam=5, dyn_path=4, k_max=200, capacity=64 * s.n_spheres)
    a = _run(dem, s, 1500, True, **kw)
    b = _run(dem, s, 1500, False, **kw)
    print(f"{mode} k={k}: {a[2].size} pairs, {_touching(a)} with history, cds {a[0]['cds']}", flush=True)
    assert a[2].size > 0
    _same(a, b)


@pytest.mark.parametrize("k", [10, 20])
def test_spinning_clumps_skipping_changes_nothing(dem, k):
    """Clumps that barely translate but spin at up to a few hundred rad/s:
    their spheres sweep towards their neighbours at ~|w| arm, many times
    their owners' speed, so a reach that left the rotation out would skip
    pairs that come to touch within a chain."""
    s = W.small_clumps(8, n=343, spacing=0.0092, vel=0.005, walls=True, gravity=(0, 0, 0), with_singles=False)
    s.W = (s.W * 12.0).astype(np.float32)
    kw = dict(mode="fixed", k=k, lam=5, dyn_path=4, capacity=64 * s.n_spheres)
    a = _run(dem, s, 2000, True, **kw)
    b = _run(dem, s, 2000, False, **kw)
    print(f"k={k}: {a[2].size} pairs, {_touching(a)} with history, cds {a[0]['cds']}", flush=True)
    assert _touching(a) > 0
    _same(a, b)


def test_clump_skipping_split_equals_two_kernel_form(dem):
    """The two-kernel form evaluates every pair every step."""
    s = W.small_clumps(6, n=216, spacing=0.0095, vel=0.2)
    kw = dict(mode="fixed", k=20, lam=5, capacity=64 * s.n_spheres)
    a = _run(dem, s, 800, True, dyn_path=4, **kw)
    b = _run(dem, s, 800, True, dyn_path=1, **kw)
    _same(a, b)


def _cube_clumps(seed, n=216, spacing=0.0095):
    """Tri-sphere clumps, eight-sphere clumps (spheres at the corners of a
    cube) and single spheres: an owner of more than six spheres takes the
    split step's path whose list entry holds no per-sphere lengths."""
    rng = np.random.default_rng(seed)
    side = int(math.ceil(n ** (1 / 3)))
    base = W.lattice((side, side, side), spacing, -0.5 * (side - 1) * spacing * np.ones(3), n_take=n)
    base = base + rng.uniform(-0.0004, 0.0004, size=(n, 3))
    q = W.random_quaternions(rng, n)
    V = rng.normal(0.0, 0.2, size=(n, 3))
    Wb = rng.normal(0.0, 20.0, size=(n, 3))
    types = rng.integers(-1, 2, size=n).astype(np.int32)
    q[types < 0] = np.array([1.0, 0, 0, 0])
    corner = 0.0017 * np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], dtype=np.float64)
    cube = (corner.astype(np.float32), np.full(8, 0.0019, dtype=np.float32))
    half = 0.5 * side * spacing + 0.006
    lo, hi = -half * np.ones(3), half * np.ones(3)
    walls = W.box_walls(lo, hi, moving={0: (0.1, 0.0, 0.0)})
    return W.assemble(types, base, q, V, Wb, [W.tri_template(0.003, 0.002), cube], 0.0025, [0, 0],
                      W.concat_walls(walls), W.materials(), (0, 0, -9.81), 5e-6, 0.0002, lo, hi,
                      name=f"cube_clumps{seed}")


def test_eight_sphere_clumps_split_equals_two_kernel_form(dem):
    """Owners of eight spheres in the split step: their bounds are read per
    sphere, the others' from their list entries; both forms end bit for
    bit in the same state, set and history."""
    s = _cube_clumps(7)
    sph0 = np.asarray(s.own_sph0)
    assert int(np.max(np.diff(sph0))) == 8
    kw = dict(mode="fixed", k=10, lam=5, capacity=64 * s.n_spheres)
    a = _run(dem, s, 1500, True, dyn_path=4, **kw)
    b = _run(dem, s, 1500, True, dyn_path=1, **kw)
    # touching pairs with a sphere of an eight-sphere owner
    keys, hist = a[2], a[3]
    touch = np.any(hist[:, :3] != 0.0, axis=1)
    big = np.diff(sph0) == 8

    def of_big(sph):
        return big[np.searchsorted(sph0, sph, side="right") - 1]

    i = (keys >> np.uint64(32)).astype(np.int64)
    j = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    jb = np.zeros_like(i, dtype=bool)
    jb[j < s.n_spheres] = of_big(j[j < s.n_spheres])
    n_big = int(np.count_nonzero(touch & (of_big(i) | jb)))
    print(f"{keys.size} pairs, {_touching(a)} with history ({n_big} with an eight-sphere clump), "
          f"cds {a[0]['cds']}", flush=True)
    assert n_big > 0
    _same(a, b)
