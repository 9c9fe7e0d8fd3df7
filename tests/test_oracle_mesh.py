"""Pins of the oracle's sphere-facet path (rigid triangle meshes with
prescribed motion; a facet is a geometry of the mesh owner, Sec. 2.4).

* the closest point of a facet against a dense sampling of the facet;
* the mesh pose against scipy's rotation-vector formula;
* a floor made of two facets against a plane floor: the same contacts and,
  for a sphere over the inside of a facet, the same force (two independent
  code paths in the oracle);
* a vertex contact against the closed-form Hertz force;
* a sphere released at rest on a floor mesh that translates at v: friction
  brings it to rolling at 2/7 v (the belt form of the 5/7 sliding law).
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import workloads as W

def _brute_closest(a, b, c, p, n=400):
    u, v = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1))
    keep = u + v <= 1.0
    u, v = u[keep], v[keep]
    pts = a[None] + u[:, None] * (b - a)[None] + v[:, None] * (c - a)[None]
    d = np.linalg.norm(pts - p[None], axis=1)
    k = np.argmin(d)
    return pts[k], d[k]


def test_closest_point_matches_dense_sampling():
    rng = np.random.default_rng(0)
    for _ in range(200):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2.0
        q = oracle.tri_closest(a, b, c, p)
        qb, db = _brute_closest(a, b, c, p)
        d = np.linalg.norm(p - q)
        # the exact closest point is never farther than the best sample, and
        # the best sample is within the sampling step of it
        assert d <= db + 1e-12
        h = 2.0 * max(np.linalg.norm(b - a), np.linalg.norm(c - a), np.linalg.norm(c - b)) / 400
        assert np.linalg.norm(q - qb) <= h
        # q lies in the triangle: barycentric coordinates in [0, 1]
        M = np.c_[b - a, c - a]
        uv, *_ = np.linalg.lstsq(M, q - a, rcond=None)
        assert uv.min() >= -1e-9 and uv.sum() <= 1 + 1e-9


def test_closest_point_of_an_interior_projection_is_the_plane_projection():
    rng = np.random.default_rng(1)
    for _ in range(100):
        a, b, c = rng.normal(size=(3, 3))
        u, v = rng.uniform(0.05, 0.45, size=2)
        inside = a + u * (b - a) + v * (c - a)
        nrm = np.cross(b - a, c - a)
        nrm /= np.linalg.norm(nrm)
        p = inside + rng.normal() * nrm
        np.testing.assert_allclose(oracle.tri_closest(a, b, c, p), inside, atol=1e-12)


def _one_sphere(z, r=0.01, floor="plane", vel=(0, 0, 0), mu=0.5, x=(0.0, 0.0)):
    L = 0.5
    X = np.array([[x[0], x[1], z]])
    if floor == "plane":
        walls = W.concat_walls(W.plane((0, 0, 0), (0, 0, 1), vel=vel))
    else:
        walls = W.concat_walls()
    s = W.assemble(np.full(1, -1), X, W._qid(1), np.zeros((1, 3)), np.zeros((1, 3)), [], r, None, walls,
                   W.materials(mu=mu), (0, 0, -9.81), 1e-6, 0.0, -np.ones(3), np.ones(3))
    if floor == "mesh":
        tri = W.quad_grid((-L, -L, 0.0), (2 * L, 0, 0), (0, 2 * L, 0), 1, 1)
        W.add_meshes(s, dict(tri=tri, origin=(0, 0, 0), vel=vel))
    return s


@pytest.mark.parametrize("delta", [1e-6, 1e-5, 1e-4])
def test_facet_floor_force_equals_plane_floor_force(delta):
    r = 0.01
    sp = _one_sphere(r - delta, r, "plane", x=(0.1, -0.2))
    sm = _one_sphere(r - delta, r, "mesh", x=(0.1, -0.2))
    op, om = oracle.Oracle(sp), oracle.Oracle(sm)
    kp, km = op.detect(op.state(), 0.0), om.detect(om.state(), 0.0)
    assert kp.size == 1 and km.size == 1
    fp = op.forces(op.state(), kp, np.zeros((1, 4)))
    fm = om.forces(om.state(), km, np.zeros((1, 4)))
    # the facet normal comes from a closest point, so its tangential parts
    # are rounding (relative 1e-15 of the force), not exact zeros
    np.testing.assert_allclose(fm["Fc"], fp["Fc"], rtol=1e-12, atol=1e-12 * abs(fp["Fc"][0, 2]))
    # static Hertz: F = 4/3 E* sqrt(r) delta^1.5 (E* of two equal materials)
    E, nu = float(sm.mat_E[0]), float(sm.mat_nu[0])
    Es = 1.0 / (2 * (1 - nu * nu) / E)
    d = float(sm.sph_rad[0]) - float(sm.X[0, 2])
    np.testing.assert_allclose(fm["Fc"][0, 2], 4.0 / 3.0 * Es * np.sqrt(float(sm.sph_rad[0])) * d ** 1.5, rtol=1e-12)


def test_vertex_contact_is_a_hertz_contact_along_the_vertex_normal():
    r = 0.01
    s = _one_sphere(0.5, r, "mesh")
    # a single facet whose vertex (0, 0, 0) is closest to the sphere
    s.tri_local = np.array([[0, 0, 0, -0.1, 0, 0, 0, -0.1, 0]], dtype=np.float64)
    s.tri_mesh = np.zeros(1, dtype=np.int32)
    dirn = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)
    d = r - 2e-5
    s.X = W.snap_pos(dirn[None] * d)
    o = oracle.Oracle(s)
    st = o.state()
    k = o.detect(st, 0.0)
    assert k.size == 1
    f = o.forces(st, k, np.zeros((1, 4)))
    x = st["X"][0]
    dd = np.linalg.norm(x)
    E, nu = float(s.mat_E[0]), float(s.mat_nu[0])
    Es = 1.0 / (2 * (1 - nu * nu) / E)
    rr = float(s.sph_rad[0])
    F = 4.0 / 3.0 * Es * np.sqrt(rr) * (rr - dd) ** 1.5
    np.testing.assert_allclose(f["Fc"][0], F * x / dd, rtol=1e-9)


def test_mesh_pose_matches_rotation_vector():
    s = W.small_mixer(0, n=8)
    o = oracle.Oracle(s)
    for step in (0, 1, 1000, 123457):
        p, R = o.mesh_pose(0, step)
        t = step * s.dt
        ref = Rotation.from_rotvec(s.mesh_omega[0] * t).as_matrix()
        np.testing.assert_allclose(R, ref, atol=1e-14)
        np.testing.assert_allclose(p, s.mesh_origin[0] + s.mesh_vel[0] * t, atol=1e-16)
    fp = o.facet_positions(1000)
    p, R = o.mesh_pose(0, 1000)
    ref = p[None] + s.tri_local.reshape(-1, 3) @ R.T
    np.testing.assert_allclose(fp.reshape(-1, 3), ref, atol=1e-15)


def test_facet_floor_contacts_match_plane_floor_contacts():
    rng = np.random.default_rng(3)
    n = 300
    X = np.c_[rng.uniform(-0.3, 0.3, size=(n, 2)), rng.uniform(0.0, 0.02, size=n)]
    r = 0.01
    mk = lambda floor: W.assemble(np.full(n, -1), X, W._qid(n), np.zeros((n, 3)), np.zeros((n, 3)), [], r, None,
                                  W.concat_walls(W.plane((0, 0, 0), (0, 0, 1))) if floor == "plane"
                                  else W.concat_walls(), W.materials(), (0, 0, -9.81), 1e-6, 0.0003,
                                  -np.ones(3), np.ones(3))
    sp, sm = mk("plane"), mk("mesh")
    W.add_meshes(sm, dict(tri=W.quad_grid((-0.5, -0.5, 0.0), (1, 0, 0), (0, 1, 0), 1, 1)))
    for m in (0.0, 0.0003):
        kp = oracle.Oracle(sp).detect(oracle.Oracle(sp).state(), m)
        km = oracle.Oracle(sm).detect(oracle.Oracle(sm).state(), m)
        jp = (kp & np.uint64(0xFFFFFFFF)).astype(np.int64)
        jm = (km & np.uint64(0xFFFFFFFF)).astype(np.int64)
        sph_p = np.unique((kp >> np.uint64(32))[jp >= n])
        sph_m = np.unique((km >> np.uint64(32))[jm >= n])
        np.testing.assert_array_equal(sph_p, sph_m)
        assert sph_p.size > 20


def test_sphere_on_a_moving_facet_floor_rolls_at_two_sevenths():
    """Released at rest on a floor translating at v, the sphere slides until
    friction makes it roll: then its speed is 2/7 v (the contact point moves
    with the floor)."""
    r, vb = 0.01, 0.05
    s = _one_sphere(r - 5e-6, r, "mesh", vel=(vb, 0, 0), mu=0.3)
    s.dt = 2e-6
    o = oracle.Oracle(s)
    st = o.state()
    # sliding lasts 2 v / (7 mu g) = 4.9 ms; run 20 ms
    st, acs, stats, step = o.run(st, 10000, mode="every")
    vx = st["V"][0, 0]
    assert abs(vx - 2.0 / 7.0 * vb) <= 0.02 * 2.0 / 7.0 * vb, vx


def test_sphere_on_a_spinning_facet_floor_is_dragged_along_omega_cross_r():
    """On a floor spinning at w about z, a sphere at rest at radius rho first
    slides: friction accelerates it at mu g along w x rho."""
    r, w, rho, mu = 0.01, 2.0, 0.2, 0.3
    s = _one_sphere(r - 5e-6, r, "mesh", mu=mu, x=(rho, 0.0))
    s.mesh_omega = np.array([[0.0, 0.0, w]])
    s.dt = 2e-6
    o = oracle.Oracle(s)
    st, acs, stats, step = o.run(o.state(), 1000, mode="every")
    t = 1000 * s.dt
    v = st["V"][0]
    assert abs(v[1] - mu * 9.81 * t) <= 0.05 * mu * 9.81 * t, v
    assert abs(v[0]) <= 0.05 * abs(v[1]), v
