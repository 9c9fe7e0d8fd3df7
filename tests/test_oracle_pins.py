"""Pins of the FP64 oracle against what the physics and the paper fix.

None of these compares the oracle with itself: each checks a closed form, a
conservation law, a library routine, a value printed in the paper, or a
brute-force enumeration.  They run on the CPU only.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


def two_spheres(x0, x1, v0, v1, r0=0.005, r1=0.005, cor=0.6, mu=0.0, dt=1e-7, E=1e8, nu=0.3,
                mats=None, mat=(0, 0), w=None):
    mats = mats or W.materials(E=E, nu=nu, cor=cor, mu=mu)
    s = W.assemble(np.full(2, -1), np.array([x0, x1]), W._qid(2), np.array([v0, v1]),
                   np.zeros((2, 3)) if w is None else w, [], np.array([r0, r1]), None,
                   W.concat_walls(), mats, (0, 0, 0), dt, 0.0, -0.5 * np.ones(3), 0.5 * np.ones(3))
    s.sph_mat[:] = mat
    return s


def collide(v, cor, dt=1e-7, r=0.005):
    """Head-on collision of two equal spheres approaching at relative speed v."""
    gap = 1e-6
    s = two_spheres([-r - gap, 0, 0], [r + gap, 0, 0], [v / 2, 0, 0], [-v / 2, 0, 0], cor=cor, dt=dt)
    o = oracle.Oracle(s)
    st = o.state()
    acs, step, dmax, t_in, t_out = None, 0, 0.0, None, None
    for _ in range(200000):
        st, acs, _, step = o.run(st, 10, mode="every", acs=acs, step=step)
        ov = 2 * r - np.linalg.norm(st["X"][0] - st["X"][1])
        dmax = max(dmax, ov)
        if ov > 0 and t_in is None:
            t_in = step
        if t_in is not None and ov < 0:
            t_out = step
            break
    e = (st["V"][1, 0] - st["V"][0, 0]) / v
    return s, e, dmax, (t_out - t_in) * dt


def test_effective_moduli_golden():
    E, nu, Es, Gs = _golden("hertz_moduli.txt")[0]
    # a static overlap with zero velocity exposes E* through the Hertz law
    r, d = 0.005, 2e-5
    s = two_spheres([0, 0, 0], [2 * r - d, 0, 0], [0, 0, 0], [0, 0, 0], E=E, nu=nu)
    o = oracle.Oracle(s)
    out = o.forces(o.state(), np.array([1], dtype=np.uint64), np.zeros((1, 3)))
    r = s.sph_rad[0]
    d = 2 * r - abs(s.X[1, 0] - s.X[0, 0])
    Rb = r / 2
    expect = 4.0 / 3.0 * Es * math.sqrt(Rb) * d ** 1.5
    assert abs(np.linalg.norm(out["Fc"][0]) - expect) <= 1e-12 * expect


@pytest.mark.parametrize("r0,r1,E0,E1,nu0,nu1", [
    (0.005, 0.005, 1e8, 1e8, 0.3, 0.3),
    (0.002, 0.006, 1e8, 1e9, 0.3, 0.25),
    (0.01, 0.003, 7e7, 2e8, 0.45, 0.2),
])
def test_hertz_static_closed_form(r0, r1, E0, E1, nu0, nu1):
    """At zero velocity the normal force is Hertz's (4/3) E* sqrt(R) d^1.5,
    along the centre line, equal and opposite (Sec. 4.1, Eq. (1))."""
    mats = dict(mat_E=np.array([E0, E1]), mat_nu=np.array([nu0, nu1]),
                mat_cor=np.full((2, 2), 0.5), mat_mu=np.full((2, 2), 0.3), mat_crr=np.zeros((2, 2)))
    d = 3e-6
    dirn = np.array([0.3, -0.5, 0.8])
    dirn /= np.linalg.norm(dirn)
    x1 = W.snap_pos((r0 + r1 - d) * dirn)
    s = two_spheres([0, 0, 0], x1, [0, 0, 0], [0, 0, 0], r0=r0, r1=r1, mats=mats, mat=(0, 1))
    o = oracle.Oracle(s)
    st = o.state()
    out = o.forces(st, np.array([1], dtype=np.uint64), np.zeros((1, 3)))
    r0, r1 = s.sph_rad
    dd = r0 + r1 - np.linalg.norm(s.X[1] - s.X[0])
    Es = 1.0 / ((1 - nu0 ** 2) / E0 + (1 - nu1 ** 2) / E1)
    Rb = r0 * r1 / (r0 + r1)
    expect = 4.0 / 3.0 * Es * math.sqrt(Rb) * dd ** 1.5
    F = out["Fc"][0]
    assert abs(np.linalg.norm(F) - expect) <= 1e-10 * expect
    # force on A (sphere 0) points from B to A
    assert np.dot(F, -x1) > 0 and np.linalg.norm(np.cross(F, x1)) <= 1e-10 * expect * np.linalg.norm(x1)
    np.testing.assert_allclose(out["Fo"][0], -out["Fo"][1], rtol=0, atol=1e-15 * expect)


def test_plane_static_closed_form():
    """Sphere on a plane: R = r, Hertz force along the plane normal."""
    r, d = 0.004, 5e-6
    s = W.assemble(np.full(1, -1), np.array([[0.0, 0.0, r - d]]), W._qid(1), np.zeros((1, 3)),
                   np.zeros((1, 3)), [], r, None, W.plane((0, 0, 0), (0, 0, 1)), W.materials(),
                   (0, 0, 0), 1e-6, 0.0, -np.ones(3), np.ones(3))
    o = oracle.Oracle(s)
    out = o.forces(o.state(), np.array([1], dtype=np.uint64), np.zeros((1, 3)))
    r = s.sph_rad[0]
    dd = r - s.X[0, 2]
    Es = 1e8 / (2 * (1 - 0.09))
    expect = 4.0 / 3.0 * Es * math.sqrt(r) * dd ** 1.5
    np.testing.assert_allclose(out["Fc"][0], [0, 0, expect], rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(out["Fw"][0], [0, 0, -expect], rtol=1e-12, atol=1e-18)


def test_elastic_collision_hertz_closed_forms():
    """CoR = 1: restitution 1, maximum overlap (15 m v^2 / (16 E* sqrt R))^(2/5)
    and contact time 2.868 (m^2 / (E*^2 R v))^(1/5) (Hertz impact theory)."""
    v = 1.0
    s, e, dmax, tc = collide(v, cor=1.0, dt=2e-8)
    m = s.own_mass[0] / 2
    Rb = s.sph_rad[0] / 2
    Es = 1e8 / (2 * (1 - 0.09))
    dmax_th = (15 * m * v * v / (16 * Es * math.sqrt(Rb))) ** 0.4
    tc_th = 2.8683 * (m * m / (Es * Es * Rb * v)) ** 0.2
    assert abs(e - 1.0) < 1e-4
    assert abs(dmax - dmax_th) / dmax_th < 2e-3
    assert abs(tc - tc_th) / tc_th < 5e-3


def test_damped_restitution_matches_cor_at_all_speeds():
    """The damping constants are inferred from CoR (Sec. 4.1): the measured
    restitution equals CoR and, because the damping scales with delta^(1/4),
    does not depend on the impact speed."""
    es = [collide(v, cor=0.6, dt=5e-8)[1] for v in (0.1, 1.0, 10.0)]
    assert max(es) - min(es) < 2e-4
    assert all(abs(e - 0.6) < 1e-3 for e in es)
    e3 = collide(1.0, cor=0.3, dt=5e-8)[1]
    assert abs(e3 - 0.3) < 1e-3


def sphere_on_plane(v0, w0, mu, gvec, r=0.005, m=None, dt=1e-6, E=1e8):
    mass = 2600 * 4 / 3 * math.pi * r ** 3 if m is None else m
    Es = E / (2 * (1 - 0.09))
    gmag = np.linalg.norm(gvec)
    deq = (mass * abs(gvec[2]) / (4 / 3 * Es * math.sqrt(r))) ** (2 / 3) if gvec[2] else 0.0
    s = W.assemble(np.full(1, -1), np.array([[0.0, 0.0, r - deq]]), W._qid(1),
                   np.array([v0]), np.array([w0]), [], r, None, W.plane((0, 0, 0), (0, 0, 1)),
                   W.materials(E=E, mu=mu), gvec, dt, 0.0, -np.ones(3), np.ones(3),
                   single_mass=np.array([mass]), single_moi=np.array([0.4 * mass * r * r]))
    return s


def test_sliding_sphere_reaches_five_sevenths():
    """A sphere launched sliding without spin on a plane ends up rolling at
    (5/7) v0, reached at t = 2 v0 / (7 mu g) (rigid-body mechanics)."""
    v0, mu, g = 0.5, 0.5, 9.81
    s = sphere_on_plane([v0, 0, 0], [0, 0, 0], mu, (0, 0, -g))
    o = oracle.Oracle(s)
    st = o.state()
    t_roll = 2 * v0 / (7 * mu * g)
    n1 = int(0.5 * t_roll / s.dt)
    st, acs, _, step = o.run(st, n1, mode="every")
    # during sliding, friction decelerates at mu g
    assert abs(st["V"][0, 0] - (v0 - mu * g * n1 * s.dt)) < 0.01 * v0
    st, acs, _, step = o.run(st, int(1.5 * t_roll / s.dt), mode="every", acs=acs, step=step)
    v = st["V"][0, 0]
    wy = st["W"][0, 1]   # spheres keep identity orientation only approximately; use world frame
    R = Rotation.from_quat(st["q"][0, [1, 2, 3, 0]]).as_matrix()
    ww = R @ st["W"][0]
    assert abs(v - 5 / 7 * v0) < 5e-3 * v0
    assert abs(v - ww[1] * s.sph_rad[0]) < 5e-3 * v0
    del wy


@pytest.mark.parametrize("alpha_deg,rolls", [(30.0, True), (39.0, True), (44.0, False), (55.0, False)])
def test_incline_rolling_threshold(alpha_deg, rolls):
    """Sec. 4.3.1: the sphere (r = 0.2 m, 5 kg, v0 = 0.5 m/s up the slope,
    mu = 0.25) rolls without sliding iff tan(alpha) <= 3.5 mu."""
    mu, crr, alpha_c, _ = _golden("incline_rolling_threshold.txt")[0]
    assert abs(math.degrees(math.atan(3.5 * mu - 2.5 * crr)) - alpha_c) < 1e-9
    a = math.radians(alpha_deg)
    g = 9.81
    gvec = (g * math.sin(a), 0.0, -g * math.cos(a))   # slope tilted about y; down-slope is +x
    s = sphere_on_plane([-0.5, 0, 0], [0, 0, 0], mu, gvec, r=0.2, m=5.0, dt=2e-5)
    o = oracle.Oracle(s)
    st, acs, _, step = o.run(o.state(), 20000, mode="every")
    v = st["V"][0, 0]
    R = Rotation.from_quat(st["q"][0, [1, 2, 3, 0]]).as_matrix()
    ww = R @ st["W"][0]
    slip = v - ww[1] * 0.2
    if rolls:
        assert abs(slip) < 2e-3 * abs(v)
    else:
        assert abs(slip) > 0.05 * abs(v)


@pytest.mark.parametrize("alpha_deg,mode", [(2.0, "stationary"), (5.0, "rolling"), (30.0, "rolling"),
                                            (42.0, "sliding")])
def test_incline_with_rolling_resistance(alpha_deg, mode):
    """Sec. 4.3.1 with C_r > 0: at rest iff tan(alpha) <= C_r, rolling
    without sliding iff tan(alpha) <= 3.5 mu - 2.5 C_r, sliding above."""
    mu, crr, alpha_roll, alpha_rest = _golden("incline_rolling_threshold.txt")[1]
    assert abs(math.degrees(math.atan(3.5 * mu - 2.5 * crr)) - alpha_roll) < 1e-9
    assert abs(math.degrees(math.atan(crr)) - alpha_rest) < 1e-9
    a = math.radians(alpha_deg)
    g = 9.81
    gvec = (g * math.sin(a), 0.0, -g * math.cos(a))
    s = sphere_on_plane([-0.5, 0, 0], [0, 0, 0], mu, gvec, r=0.2, m=5.0, dt=2e-5)
    s.mat_crr[:] = crr
    o = oracle.Oracle(s)
    st, acs, _, step = o.run(o.state(), 40000, mode="every")
    v = st["V"][0, 0]
    R = Rotation.from_quat(st["q"][0, [1, 2, 3, 0]]).as_matrix()
    slip = v - (R @ st["W"][0])[1] * 0.2
    if mode == "stationary":
        assert abs(v) < 1e-3
        st2, *_ = o.run(st, 5000, mode="every", acs=acs, step=step)
        assert abs(st2["X"][0, 0] - st["X"][0, 0]) < 1e-4
    elif mode == "rolling":
        assert v > 0.05 and abs(slip) < 2e-3 * v
    else:
        assert abs(slip) > 0.05 * abs(v)


def test_torque_free_spin_closed_form():
    """No contacts, no gravity: q(t) = q0 (x) exp(t w / 2) for constant body
    angular velocity w (isotropic inertia)."""
    rng = np.random.default_rng(3)
    n = 5
    q0 = W.random_quaternions(rng, n)
    w = W.f32(rng.normal(0, 30, size=(n, 3)))
    X = W.snap_pos(np.arange(n)[:, None] * np.array([0.1, 0, 0]))
    s = W.assemble(np.full(n, -1), X, q0, np.zeros((n, 3)), w, [], 0.01, None, W.concat_walls(),
                   W.materials(), (0, 0, 0), 1e-4, 0.0, -np.ones(3), np.ones(3))
    o = oracle.Oracle(s)
    steps = 1000
    st, *_ = o.run(o.state(), steps, mode="every")
    t = steps * s.dt
    for i in range(n):
        R0 = Rotation.from_quat(q0[i, [1, 2, 3, 0]])
        Rt = R0 * Rotation.from_rotvec(w[i] * t)
        got = Rotation.from_quat(st["q"][i, [1, 2, 3, 0]])
        assert (got.inv() * Rt).magnitude() < 1e-10
        np.testing.assert_array_equal(st["W"][i], w[i])


def test_sphere_centres_match_library_rotation():
    s = W.small_clumps(5, n=40)
    o = oracle.Oracle(s)
    xs = o.sphere_centres(o.state())
    R = Rotation.from_quat(s.q[:, [1, 2, 3, 0]]).as_matrix()
    expect = s.X[s.sph_owner] + np.einsum("nij,nj->ni", R[s.sph_owner], s.sph_local)
    np.testing.assert_allclose(xs, expect, rtol=0, atol=1e-15)


def _momentum(s, st):
    return (s.own_mass[:, None] * st["V"]).sum(0)


def _angular_momentum(s, st):
    R = Rotation.from_quat(st["q"][:, [1, 2, 3, 0]]).as_matrix()
    spin = np.einsum("nij,nj->ni", R, s.own_moi * st["W"])
    return (s.own_mass[:, None] * np.cross(st["X"], st["V"])).sum(0) + spin.sum(0)


def test_linear_momentum_conserved_with_clumps():
    """No walls, no gravity: contact forces come in equal and opposite pairs
    (third law), so total momentum is conserved to rounding."""
    s = W.small_clumps(11, n=64, vel=0.5, walls=False, gravity=(0, 0, 0), with_singles=True)
    o = oracle.Oracle(s)
    st = o.state()
    p0 = _momentum(s, st)
    st, acs, stats, _ = o.run(st, 400, mode="every")
    assert stats["sum_acs"] > 100
    scale = (s.own_mass[:, None] * np.abs(s.V)).sum()
    assert np.abs(_momentum(s, st) - p0).max() < 1e-12 * scale


def test_angular_momentum_conserved_spheres():
    """For spheres (isotropic inertia) the semi-implicit update conserves
    total angular momentum about the origin exactly in exact arithmetic."""
    s = W.small_spheres(12, n=150, vel=0.5, walls=False, gravity=(0, 0, 0))
    o = oracle.Oracle(s)
    st = o.state()
    L0 = _angular_momentum(s, st)
    st, acs, stats, _ = o.run(st, 400, mode="every")
    assert stats["sum_acs"] > 100
    scale = np.abs(s.own_mass[:, None] * np.cross(s.X, s.V)).sum() + np.abs(s.own_moi * s.W).sum()
    assert np.abs(_angular_momentum(s, st) - L0).max() < 1e-11 * scale


def _energy(s, o, st, step):
    ke = 0.5 * (s.own_mass * (st["V"] ** 2).sum(1)).sum() + 0.5 * (s.own_moi * st["W"] ** 2).sum()
    pe = -(s.own_mass[:, None] * st["X"] * s.gravity).sum()
    keys = o.detect(st, 0.0, step=step)
    xs = o.sphere_centres(st)
    Es = 1e8 / (2 * (1 - 0.09))
    el = 0.0
    wp = o.wall_positions(step)
    for k in keys:
        i, j = int(k >> 32), int(k & 0xFFFFFFFF)
        if j < s.n_spheres:
            d = s.sph_rad[i] + s.sph_rad[j] - np.linalg.norm(xs[i] - xs[j])
            Rb = s.sph_rad[i] * s.sph_rad[j] / (s.sph_rad[i] + s.sph_rad[j])
        else:
            w = j - s.n_spheres
            d = s.sph_rad[i] - np.dot(xs[i] - wp[w], s.wall_geom[w, 3:6])
            Rb = s.sph_rad[i]
        el += 8.0 / 15.0 * Es * math.sqrt(Rb) * d ** 2.5
    return ke + pe + el


@pytest.mark.parametrize("clumps", [False, True])
def test_energy_conserved_without_dissipation(clumps):
    """CoR = 1 and mu = 0: kinetic + gravitational + Hertz elastic energy
    ((8/15) E* sqrt(R) delta^(5/2)) drifts only at O(h)."""
    if clumps:
        s = W.small_clumps(21, n=27, vel=0.3, dt=2e-6, spacing=0.0115, jitter=0.0003)
    else:
        s = W.small_spheres(21, n=64, vel=0.3, dt=2e-6, gap=0.0012, jitter=0.0004)
    for k in ("mat_cor",):
        getattr(s, k)[:] = 1.0
    s.mat_mu[:] = 0.0
    s.wall_vel[:] = 0.0
    drifts = []
    for dt in (2e-6, 1e-6):
        s.dt = dt
        o = oracle.Oracle(s)
        st = o.state()
        E0 = _energy(s, o, st, 0)
        n = int(round(8e-3 / dt))
        st, acs, stats, step = o.run(st, n, mode="every")
        assert stats["sum_acs"] > 0
        drifts.append(abs(_energy(s, o, st, step) - E0))
    ke0 = 0.5 * (s.own_mass * (s.V ** 2).sum(1)).sum()
    assert drifts[0] < 2e-3 * ke0
    assert drifts[1] < 0.7 * drifts[0] + 1e-12 * ke0


def test_static_pile_force_balance():
    """After settling, the walls carry the weight of the pile (side walls
    take a share through friction) and each sphere is in force balance
    (Eq. (3) at rest)."""
    rng = np.random.default_rng(4)
    n = 27
    base = W.lattice((3, 3, 3), 0.0105, np.array([-0.0105, -0.0105, 0.006]))
    X = base + rng.uniform(-0.0004, 0.0004, size=(n, 3))
    lo, hi = np.array([-0.0165, -0.0165, 0.0]), np.array([0.0165, 0.0165, 0.1])
    s = W.assemble(np.full(n, -1), X, W._qid(n), np.zeros((n, 3)), np.zeros((n, 3)), [], 0.005,
                   None, W.box_walls(lo, hi), W.materials(cor=0.2, mu=0.5), (0, 0, -9.81), 1e-5, 0.0,
                   lo, hi)
    o = oracle.Oracle(s)
    st, acs, _, step = o.run(o.state(), 60000, mode="every")
    out = o.forces(st, acs[0], acs[1], step=step)
    M = s.own_mass.sum()
    walls = out["Fw"].sum(0)
    assert abs(-walls[2] - M * 9.81) < 1e-3 * M * 9.81
    assert np.abs(walls[:2]).max() < 1e-3 * M * 9.81
    assert -out["Fw"][4][2] > 0.5 * M * 9.81
    resid = np.linalg.norm(out["Fo"] + s.own_mass[:, None] * s.gravity, axis=1)
    assert resid.max() < 1e-3 * s.own_mass.max() * 9.81


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("margin", [0.0, 0.0002, 0.001])
def test_binned_detection_equals_brute_force(seed, margin):
    """Binned contact detection returns exactly the O(N^2) enumeration."""
    sp = W.small_spheres(seed, n=300)
    cl = W.small_clumps(seed, n=100, with_cylinder=True)
    for s in (sp, cl):
        o = oracle.Oracle(s)
        st = o.state()
        a = o.detect(st, margin, brute=True)
        b = o.detect(st, margin)
        assert a.size > 0
        np.testing.assert_array_equal(a, b)
        assert np.all(np.diff(a.astype(np.float64)) > 0)


def test_brute_force_matches_numpy_pairwise():
    """The brute-force predicate equals a direct numpy pairwise test."""
    s = W.small_spheres(3, n=120, walls=False)
    o = oracle.Oracle(s)
    st = o.state()
    m = 0.0003
    got = o.detect(st, m, brute=True)
    x = s.X
    d2 = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    T = s.sph_rad[:, None] + s.sph_rad[None, :] + 2 * m
    ii, jj = np.nonzero(np.triu(d2 < T * T, 1))
    exp = (ii.astype(np.uint64) << np.uint64(32)) | jj.astype(np.uint64)
    np.testing.assert_array_equal(got, np.sort(exp))


def test_coulomb_cap_holds_every_contact():
    s = W.small_clumps(8, n=64, vel=0.8)
    o = oracle.Oracle(s)
    st = o.state()
    keys = o.detect(st, 0.0)
    rng = np.random.default_rng(1)
    hist = rng.normal(0, 2e-5, size=(keys.size, 3))
    out = o.forces(st, keys, hist)
    xs = o.sphere_centres(st)
    wp = o.wall_positions(0)
    for c, k in enumerate(keys):
        i, j = int(k >> 32), int(k & 0xFFFFFFFF)
        if j < s.n_spheres:
            n = xs[i] - xs[j]
        elif s.wall_type[j - s.n_spheres] == 0:
            n = s.wall_geom[j - s.n_spheres, 3:6].copy()
        else:
            continue
        n /= np.linalg.norm(n)
        F = out["Fc"][c]
        Fn = np.dot(F, n) * n
        Ft = F - Fn
        assert np.linalg.norm(Ft) <= 0.5 * np.linalg.norm(Fn) * (1 + 1e-9) + 1e-15


def test_delayed_detection_equals_every_step_bitwise():
    """Sec. 2.1: with a margin that covers the motion between updates, the
    delayed set contains every true contact; false positives give exactly
    zero force, so the trajectory equals every-step detection bit for bit."""
    s = W.small_spheres(9, n=125, vel=0.3)
    o = oracle.Oracle(s)
    a, acs_a, st_a, _ = o.run(o.state(), 300, mode="every")
    b, acs_b, st_b, _ = o.run(o.state(), 300, mode="fixed", k=10, lam=5, margin=0.0003, judge=True)
    assert st_b["misses"] == 0 and st_b["cds"] == 30
    for key in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(a[key], b[key])


def test_judge_counts_misses_and_repairs_keep_exactness():
    """A margin too thin for the interval misses contacts; the judge counts
    them and repairs the set before any force is evaluated, so the run still
    equals every-step detection bit for bit."""
    s = W.small_spheres(10, n=125, vel=1.0)
    o = oracle.Oracle(s)
    a, *_ = o.run(o.state(), 300, mode="every")
    b, acs_b, st_b, _ = o.run(o.state(), 300, mode="fixed", k=40, lam=20, margin=1e-6, judge=True)
    assert st_b["misses"] > 0 and st_b["repairs"] > 0
    for key in ("X", "q", "V", "W"):
        np.testing.assert_array_equal(a[key], b[key])


def test_history_survives_active_set_updates():
    """Sec. 4.2: a contact's history lives while the contact lives; a
    sliding pair keeps the same tangential displacement whether the set is
    rebuilt every step or every 10 steps."""
    s = sphere_on_plane([0.05, 0, 0], [0, 0, 0], 0.5, (0, 0, -9.81), dt=1e-6)
    o = oracle.Oracle(s)
    a, acs_a, _, _ = o.run(o.state(), 500, mode="every")
    b, acs_b, stats, _ = o.run(o.state(), 500, mode="fixed", k=10, lam=3, margin=1e-5, judge=True)
    assert stats["misses"] == 0
    assert np.abs(acs_a[1]).max() > 0
    np.testing.assert_array_equal(acs_a[0], acs_b[0])
    np.testing.assert_array_equal(acs_a[1], acs_b[1])


@pytest.mark.parametrize("seed", [0, 1])
def test_count_missing_equals_brute_set_difference(seed):
    """The judge's count (Sec. 2.1: every pair that touches must be in the
    set in use) equals the size of a set difference taken directly: the
    touching pairs of a brute-force O(N^2) enumeration at margin 0, minus
    the set in use, computed with numpy.  The set in use is one detected
    with a margin on an earlier state, so some pairs that touch now are
    absent from it and some pairs in it no longer touch."""
    s = W.small_clumps(seed, n=150, vel=1.5, spacing=0.0088)
    o = oracle.Oracle(s)
    st0 = o.state()
    stale = o.detect(st0, 0.00005)
    st, *_ = o.run(o.state(), 400, mode="every")
    true = o.detect(st, 0.0, brute=True)
    expect = np.setdiff1d(true, stale).size
    assert expect > 0, "the case must have missing pairs"
    assert np.setdiff1d(stale, true).size > 0
    assert o.count_missing(st, stale) == expect
    # a set holding every true pair misses nothing
    assert o.count_missing(st, np.union1d(true, stale)) == 0


def test_detect_row_equals_filtered_brute_force():
    """The one-row detection used for sampled checks of very large inputs
    equals the rows of the brute-force enumeration of the whole system."""
    s = W.small_clumps(4, n=120, with_cylinder=True, spacing=0.0085)
    o = oracle.Oracle(s)
    st = o.state()
    m = 0.0004
    brute = o.detect(st, m, brute=True)
    owners = (brute >> np.uint64(32)).astype(np.int64)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.integers(0, s.n_spheres, 40), owners[:: max(1, owners.size // 20)]]))
    got = o.detect_rows(st, m, rows)
    nonempty = 0
    for i, g in zip(rows, got):
        exp = brute[owners == i]
        np.testing.assert_array_equal(g, exp)
        nonempty += exp.size > 0
    assert nonempty >= 10
