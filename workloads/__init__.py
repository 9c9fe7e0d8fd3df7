"""Seeded synthetic DEM workloads, shared by the FP64 oracle and the HIP path.

This module only *builds inputs*: sphere/clump arrays, clump templates, walls,
materials and an initial state. It holds none of the method's arithmetic
(no contact detection, no force law, no integration).  Every array it returns
is snapped to a value that both sides can hold exactly:

* positions are multiples of 2^-36 m, so an integer voxel index plus a 32-bit
  float offset represents them without rounding, and their FP64 value is the
  same on both sides;
* velocities, angular velocities, radii, masses, inertias and template
  positions are float32-representable, because the GPU stores them as float32;
* quaternions are FP64 unit quaternions (the GPU stores them in FP64).

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in a fixed order:
radii, jitter, orientations, velocities, types.

The workloads stand in for the paper's experiments (Sec. 5, Sec. 6), whose
meshes and measured data are not available; they follow the shapes, sizes and
value ranges of the five benchmark configurations documented with the bench.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

POS_QUANTUM = 2.0 ** -36          # positions snap to this grid (metres)
VOXEL_SIZE = 2.0 ** -14           # voxel edge; offsets live in [0, VOXEL_SIZE)
RHO = 2600.0                      # particle density, kg/m^3

PLANE = 0
CYLINDER = 1


def snap_pos(x):
    return np.round(np.asarray(x, dtype=np.float64) / POS_QUANTUM) * POS_QUANTUM


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclass
class System:
    """All inputs of one DEM problem plus an initial state (host, numpy)."""
    # owners (clumps or single spheres)
    own_sph0: np.ndarray      # int32 [No+1]  spheres of owner o are sph0[o]..sph0[o+1]-1
    own_tmpl: np.ndarray      # int32 [No]    -1 = single sphere at the owner centre
    own_mass: np.ndarray      # f64   [No]
    own_moi: np.ndarray       # f64   [No,3] principal moments (template frame)
    # spheres (owner-major order; sphere id = row)
    sph_owner: np.ndarray     # int32 [Ns]
    sph_comp: np.ndarray      # int32 [Ns]   component index inside the template
    sph_local: np.ndarray     # f64   [Ns,3] position in the owner's principal frame
    sph_rad: np.ndarray       # f64   [Ns]
    sph_mat: np.ndarray       # int32 [Ns]
    # clump templates (component positions, principal frame)
    tmpl_sph0: np.ndarray     # int32 [T+1]
    tmpl_local: np.ndarray    # f64   [sum,3]
    # analytic walls with prescribed motion
    wall_type: np.ndarray     # int32 [W]  0 plane, 1 cylinder
    wall_geom: np.ndarray     # f64   [W,8] plane: p0,n ; cylinder: c,axis,R,L
    wall_vel: np.ndarray      # f64   [W,3]
    wall_omega: np.ndarray    # f64   [W,3]
    wall_mat: np.ndarray      # int32 [W]
    # materials: E, nu per material; CoR, mu, Crr per material pair
    mat_E: np.ndarray
    mat_nu: np.ndarray
    mat_cor: np.ndarray
    mat_mu: np.ndarray
    mat_crr: np.ndarray
    gravity: np.ndarray
    dt: float
    margin: float
    domain_lo: np.ndarray
    domain_hi: np.ndarray
    # initial state
    X: np.ndarray             # f64 [No,3]
    q: np.ndarray             # f64 [No,4] (w,x,y,z), body -> world
    V: np.ndarray             # f64 [No,3]
    W: np.ndarray             # f64 [No,3] angular velocity in the body frame
    name: str = ""
    meta: dict = field(default_factory=dict)
    # rigid triangle meshes with prescribed motion (Sec. 2.4: a mesh is an
    # owner, each facet a geometry): facet vertices in the mesh frame; mesh
    # frame origin at t = 0, constant velocity and angular velocity (world)
    tri_mesh: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))      # int32 [T]
    tri_local: np.ndarray = field(default_factory=lambda: np.zeros((0, 9)))               # f64 [T,9]
    mesh_origin: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))             # f64 [M,3]
    mesh_vel: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))                # f64 [M,3]
    mesh_omega: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))              # f64 [M,3]
    mesh_mat: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))     # int32 [M]
    # family tags (Sec. 2.2.2; empty = every family 0, nothing switched off):
    # per owner / wall / mesh a family 0..255; fam_pair_off[256 a + b] = 1
    # switches contacts between families a and b off; fam_fixed[a] = 1 keeps
    # the owners of family a in place
    owner_family: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))  # u8 [No]
    wall_family: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))   # u8 [W]
    mesh_family: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))   # u8 [M]
    fam_pair_off: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))  # u8 [65536]
    fam_fixed: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))     # u8 [256]

    @property
    def n_owners(self):
        return int(self.own_tmpl.shape[0])

    @property
    def n_spheres(self):
        return int(self.sph_rad.shape[0])

    @property
    def n_walls(self):
        return int(self.wall_type.shape[0])

    @property
    def n_tri(self):
        return int(self.tri_mesh.shape[0])

    @property
    def n_mesh(self):
        return int(self.mesh_mat.shape[0])

    def copy_state(self):
        return dict(X=self.X.copy(), q=self.q.copy(), V=self.V.copy(), W=self.W.copy())


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def materials(E=1e8, nu=0.3, cor=0.6, mu=0.5, crr=0.0, n=1):
    """Material table in the form the paper's LoadMaterial takes (Sec. 3):
    E and nu per material, CoR / mu / Crr per material pair."""
    return dict(mat_E=np.full(n, E), mat_nu=np.full(n, nu),
                mat_cor=np.full((n, n), cor), mat_mu=np.full((n, n), mu),
                mat_crr=np.full((n, n), crr))


def box_walls(lo, hi, mat=0, moving=None):
    """Six inward-facing planes bounding [lo, hi]; ``moving`` maps a wall index
    (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z) to a prescribed velocity."""
    lo = snap_pos(lo)
    hi = snap_pos(hi)
    geom, vel = [], []
    for ax in range(3):
        for side in (0, 1):
            p = np.zeros(3)
            n = np.zeros(3)
            p[ax] = lo[ax] if side == 0 else hi[ax]
            n[ax] = 1.0 if side == 0 else -1.0
            geom.append(np.r_[p, n, 0.0, 0.0])
            vel.append(np.zeros(3))
    if moving:
        for k, v in moving.items():
            vel[k] = np.asarray(v, dtype=np.float64)
    W = len(geom)
    return dict(wall_type=np.zeros(W, np.int32), wall_geom=np.array(geom),
                wall_vel=np.array(vel), wall_omega=np.zeros((W, 3)),
                wall_mat=np.full(W, mat, np.int32))


def concat_walls(*ws):
    if not ws:
        return dict(wall_type=np.zeros(0, np.int32), wall_geom=np.zeros((0, 8)),
                    wall_vel=np.zeros((0, 3)), wall_omega=np.zeros((0, 3)),
                    wall_mat=np.zeros(0, np.int32))
    return {k: np.concatenate([w[k] for w in ws]) for k in ws[0]}


def plane(p0, normal, vel=(0, 0, 0), mat=0):
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)
    return dict(wall_type=np.array([PLANE], np.int32),
                wall_geom=np.array([np.r_[snap_pos(p0), n, 0.0, 0.0]]),
                wall_vel=np.array([vel], dtype=np.float64),
                wall_omega=np.zeros((1, 3)), wall_mat=np.array([mat], np.int32))


def cylinder(centre, axis, radius, length, vel=(0, 0, 0), omega=(0, 0, 0), mat=0):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return dict(wall_type=np.array([CYLINDER], np.int32),
                wall_geom=np.array([np.r_[snap_pos(centre), a, radius, length]]),
                wall_vel=np.array([vel], dtype=np.float64),
                wall_omega=np.array([omega], dtype=np.float64),
                wall_mat=np.array([mat], np.int32))


def template_mass_props(local, radii, rho=RHO, n=128):
    """Mass, centroid and principal moments of a union of spheres, integrated
    on a fixed n^3 midpoint grid (the paper takes these as user input)."""
    local = np.asarray(local, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    lo = (local - radii[:, None]).min(0)
    hi = (local + radii[:, None]).max(0)
    ext = hi - lo
    step = ext / n
    ax = [lo[k] + (np.arange(n) + 0.5) * step[k] for k in range(3)]
    gx, gy, gz = np.meshgrid(*ax, indexing="ij")
    inside = np.zeros(gx.shape, dtype=bool)
    for c, r in zip(local, radii):
        inside |= (gx - c[0]) ** 2 + (gy - c[1]) ** 2 + (gz - c[2]) ** 2 < r * r
    dv = float(np.prod(step))
    x, y, z = gx[inside], gy[inside], gz[inside]
    mass = rho * dv * x.size
    cm = np.array([x.mean(), y.mean(), z.mean()])
    x, y, z = x - cm[0], y - cm[1], z - cm[2]
    Ixx = rho * dv * np.sum(y * y + z * z)
    Iyy = rho * dv * np.sum(x * x + z * z)
    Izz = rho * dv * np.sum(x * x + y * y)
    Ixy = -rho * dv * np.sum(x * y)
    Ixz = -rho * dv * np.sum(x * z)
    Iyz = -rho * dv * np.sum(y * z)
    return mass, cm, np.array([[Ixx, Ixy, Ixz], [Ixy, Iyy, Iyz], [Ixz, Iyz, Izz]])


def tri_template(r, circumradius):
    ang = np.deg2rad([90.0, 210.0, 330.0])
    loc = np.stack([circumradius * np.cos(ang), circumradius * np.sin(ang), np.zeros(3)], 1)
    return f32(loc), f32(np.full(3, r))


def penta_template(r, circumradius):
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    v *= circumradius / math.sqrt(3.0)
    loc = np.vstack([v, np.zeros((1, 3))])
    return f32(loc), f32(np.full(5, r))


def random_quaternions(rng, n):
    """Uniform random unit quaternions (Shoemake's subgroup algorithm)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([b * np.cos(2 * np.pi * u3), a * np.sin(2 * np.pi * u2),
                  a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3)], 1)
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def assemble(owner_tmpl, X, q, V, W, templates, single_rad, sph_mat_of_tmpl,
             walls, mats, gravity, dt, margin, domain_lo, domain_hi, name="",
             single_mass=None, single_moi=None, meta=None):
    """Expand owners into the owner-major sphere arrays.

    owner_tmpl: -1 for a single sphere (radius from ``single_rad``), else the
    template index. ``templates`` is a list of (local[k,3], radii[k]) in the
    template's principal frame with the centroid at the origin.
    """
    owner_tmpl = np.asarray(owner_tmpl, dtype=np.int32)
    No = owner_tmpl.shape[0]
    counts = np.ones(No, dtype=np.int64)
    tmass, tmoi = [], []
    for (loc, rad) in templates:
        m, cm, I = template_mass_props(loc, rad)
        tmass.append(float(np.float32(m)))
        tmoi.append(f32(np.diag(I)))
    for t, (loc, rad) in enumerate(templates):
        counts[owner_tmpl == t] = len(rad)
    sph0 = np.zeros(No + 1, dtype=np.int64)
    np.cumsum(counts, out=sph0[1:])
    Ns = int(sph0[-1])
    sph_owner = np.repeat(np.arange(No, dtype=np.int64), counts)
    comp = np.arange(Ns, dtype=np.int64) - sph0[sph_owner]
    sph_local = np.zeros((Ns, 3))
    sph_rad = np.zeros(Ns)
    sph_mat = np.zeros(Ns, dtype=np.int32)
    own_mass = np.zeros(No)
    own_moi = np.zeros((No, 3))
    single = owner_tmpl < 0
    if single.any():
        sidx = sph0[:-1][single]
        r = f32(np.asarray(single_rad)[single] if np.ndim(single_rad) else np.full(single.sum(), single_rad))
        sph_rad[sidx] = r
        m = f32(RHO * 4.0 / 3.0 * np.pi * r ** 3) if single_mass is None else f32(single_mass)
        own_mass[single] = m
        own_moi[single] = f32(0.4 * m * r * r)[:, None] if single_moi is None else f32(single_moi)
    tmpl_sph0 = [0]
    tmpl_local = []
    for t, (loc, rad) in enumerate(templates):
        sel = owner_tmpl == t
        tmpl_local.append(loc)
        tmpl_sph0.append(tmpl_sph0[-1] + len(rad))
        if not sel.any():
            continue
        own_mass[sel] = tmass[t]
        own_moi[sel] = tmoi[t]
        for k in range(len(rad)):
            sidx = sph0[:-1][sel] + k
            sph_local[sidx] = loc[k]
            sph_rad[sidx] = rad[k]
            sph_mat[sidx] = sph_mat_of_tmpl[t] if sph_mat_of_tmpl is not None else 0
    tmpl_local = np.vstack(tmpl_local) if tmpl_local else np.zeros((0, 3))
    return System(own_sph0=sph0.astype(np.int32), own_tmpl=owner_tmpl,
                  own_mass=own_mass, own_moi=own_moi,
                  sph_owner=sph_owner.astype(np.int32), sph_comp=comp.astype(np.int32),
                  sph_local=sph_local, sph_rad=sph_rad, sph_mat=sph_mat,
                  tmpl_sph0=np.asarray(tmpl_sph0, dtype=np.int32), tmpl_local=tmpl_local,
                  **walls, **mats,
                  gravity=np.asarray(gravity, dtype=np.float64), dt=float(dt),
                  margin=float(margin), domain_lo=snap_pos(domain_lo),
                  domain_hi=snap_pos(domain_hi),
                  X=snap_pos(X), q=np.asarray(q, dtype=np.float64),
                  V=f32(V), W=f32(W), name=name, meta=dict(meta or {}))


def lattice(counts, spacing, origin, n_take=None, order="zyx"):
    """Lattice sites filled bottom layer first (z slowest, x fastest)."""
    nx, ny, nz = counts
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], 1).astype(np.float64)
    pts = np.asarray(origin) + pts * spacing
    if n_take is not None:
        pts = pts[:n_take]
    return pts


# --------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------

def config0(seed=0):
    """1,000 monodisperse spheres (r = 5 mm) on a jittered 10^3 lattice with
    12 mm spacing inside a 0.2 m box of six planes; N(0, 0.1 m/s) velocities;
    dt = 1e-5 s, 2,000 steps; detection every step."""
    rng = np.random.default_rng(seed)
    n = 1000
    r = 0.005
    base = lattice((10, 10, 10), 0.012, -4.5 * 0.012 * np.ones(3))
    jit = rng.uniform(-0.001, 0.001, size=(n, 3))
    V = rng.normal(0.0, 0.1, size=(n, 3))
    lo, hi = -0.1 * np.ones(3), 0.1 * np.ones(3)
    return assemble(np.full(n, -1), base + jit, _qid(n), V, np.zeros((n, 3)), [], r, None,
                    box_walls(lo, hi), materials(), (0, 0, -9.81), 1e-5, 0.0, lo, hi,
                    name="config0", meta=dict(steps=2000, seed=seed))


def config1(seed=0, n=1_000_000):
    """Polydisperse spheres r ~ U(2,3) mm on a jittered lattice (7.5 mm
    spacing, bottom layers first) in a 0.6 x 0.6 x 1.2 m box, released from
    rest; dt = 5e-6 s; margin 0.1 r_min = 0.2 mm."""
    rng = np.random.default_rng(seed)
    s = 0.0075
    counts = (80, 80, 160)
    if n > counts[0] * counts[1] * counts[2]:
        raise ValueError("config1 lattice holds at most 1,024,000 spheres")
    base = lattice(counts, s, 0.5 * s * np.ones(3), n_take=n)
    rad = rng.uniform(0.002, 0.003, size=n)
    jit = rng.uniform(-0.0007, 0.0007, size=(n, 3))
    lo, hi = np.zeros(3), np.array([0.6, 0.6, 1.2])
    return assemble(np.full(n, -1), base + jit, _qid(n), np.zeros((n, 3)), np.zeros((n, 3)),
                    [], rad, None, box_walls(lo, hi), materials(), (0, 0, -9.81), 5e-6,
                    0.0002, lo, hi, name="config1", meta=dict(steps=5000, seed=seed, k=10))


def config2(seed=0, n_tri=900_000, n_penta=100_000):
    """Tri-sphere clumps (r = 3 mm, 2 mm circumradius) and five-sphere clumps
    (tetrahedron + centre, r = 2.5 mm, 2.5 mm circumradius) with uniform
    random orientations on a 10.5 mm lattice in a 1.0 x 1.0 x 1.2 m box; the
    -x wall is a plate pushing at +0.1 m/s; dt = 5e-6 s."""
    rng = np.random.default_rng(seed)
    n = n_tri + n_penta
    s = 0.0105
    counts = (95, 95, 111)
    if n > counts[0] * counts[1] * counts[2]:
        raise ValueError("config2 lattice too small")
    base = lattice(counts, s, 0.5 * s * np.ones(3) + np.array([0.0, 0.0, 0.0]), n_take=n)
    jit = rng.uniform(-0.0002, 0.0002, size=(n, 3))
    q = random_quaternions(rng, n)
    types = np.r_[np.zeros(n_tri, np.int32), np.ones(n_penta, np.int32)]
    types = types[rng.permutation(n)]
    lo, hi = np.zeros(3), np.array([1.0, 1.0, 1.2])
    walls = box_walls(lo, hi, moving={0: (0.1, 0.0, 0.0)})
    return assemble(types, base + jit, q, np.zeros((n, 3)), np.zeros((n, 3)),
                    [tri_template(0.003, 0.002), penta_template(0.0025, 0.0025)], 0.0,
                    [0, 0], walls, materials(), (0, 0, -9.81), 5e-6, 0.00025, lo, hi,
                    name="config2", meta=dict(steps=5000, seed=seed, k=10))


def config3(seed=7, n=8_000_000):
    """Granular column: lognormal radii (median 3 mm, sigma 0.25, clipped to
    [1.5, 6] mm) on a 12.5 mm lattice in a 2 x 2 m footprint (160 x 160 sites
    per layer at 8 M spheres; smaller n shrink the footprint with the cube
    root so the column keeps its aspect), released onto a floor inside far
    side walls; dt = 5e-6 s; margin 0.15 mm."""
    rng = np.random.default_rng(seed)
    s = 0.0125
    per = max(4, int(round(160 * (n / 8_000_000) ** (1.0 / 3.0))))
    layers = -(-n // (per * per))
    half = 0.5 * per * s
    base = lattice((per, per, layers), s, np.array([-half + 0.5 * s, -half + 0.5 * s, 0.5 * s]),
                   n_take=n)
    rad = np.clip(0.003 * np.exp(0.25 * rng.standard_normal(n)), 0.0015, 0.006)
    jit = rng.uniform(-0.0002, 0.0002, size=(n, 3))
    top = base[:, 2].max() + 0.02
    lo, hi = np.array([-5.0, -5.0, 0.0]), np.array([5.0, 5.0, max(top, 1.0)])
    walls = concat_walls(plane(lo, (0, 0, 1)), plane((-5.0, 0, 0), (1, 0, 0)),
                         plane((5.0, 0, 0), (-1, 0, 0)), plane((0, -5.0, 0), (0, 1, 0)),
                         plane((0, 5.0, 0), (0, -1, 0)))
    lo_dom = np.array([-1.25 * half - 0.05, -1.25 * half - 0.05, 0.0])
    hi_dom = np.array([1.25 * half + 0.05, 1.25 * half + 0.05, top])
    return assemble(np.full(n, -1), base + jit, _qid(n), np.zeros((n, 3)), np.zeros((n, 3)),
                    [], rad, None, walls, materials(), (0, 0, -9.81), 5e-6, 0.00015,
                    lo_dom, hi_dom, name="config3", meta=dict(steps=20000, seed=seed))


def config4(seed=0, n_owners=32_000_000, frac_single=18.0 / 32.0):
    """Large bed (about 60 M spheres at full size): single spheres
    (r = 2 mm) and tri-sphere clumps (r = 2 mm, circumradius 4/3 mm) on a
    7 mm lattice filling a 2 x 2 m container bottom-up (the bed is built
    packed rather than settled), then an analytic cylinder (R = 0.1 m,
    L = 0.5 m, axis y) resting on the bed top moves +x at 0.2 m/s with
    rolling angular velocity v / R; dt = 5e-6 s; margin 0.2 mm."""
    rng = np.random.default_rng(seed)
    s = 0.007
    per = max(4, int(round(285 * (n_owners / 32_000_000) ** 0.5)))
    layers = -(-n_owners // (per * per))
    half = 0.5 * per * s
    base = lattice((per, per, layers), s, np.array([-half + 0.5 * s, -half + 0.5 * s, 0.5 * s]),
                   n_take=n_owners)
    jit = rng.uniform(-0.0002, 0.0002, size=(n_owners, 3))
    q = random_quaternions(rng, n_owners)
    types = np.where(rng.random(n_owners) < frac_single, -1, 0).astype(np.int32)
    q[types < 0] = np.array([1.0, 0, 0, 0])
    top = base[:, 2].max() + 0.0035
    lo, hi = np.array([-half - 0.003, -half - 0.003, 0.0]), np.array([half + 0.003, half + 0.003, top + 0.25])
    R = 0.1
    # the cylinder starts 0.3 m in from the -x edge (on reduced beds, 5 cm
    # short of the centre, so that it always rolls on the bed)
    x0 = -half + min(0.3, half - 0.05)
    cyl = cylinder((x0, 0.0, top + R - 0.0005), (0, 1, 0), R, 0.5, vel=(0.2, 0.0, 0.0),
                   omega=(0.0, 0.2 / R, 0.0))
    walls = concat_walls(box_walls(lo, hi), cyl)
    return assemble(types, base + jit, q, np.zeros((n_owners, 3)), np.zeros((n_owners, 3)),
                    [tri_template(0.002, 0.002 * 2.0 / 3.0)], 0.002, [0], walls, materials(),
                    (0, 0, -9.81), 5e-6, 0.0002, lo, hi, name="config4",
                    meta=dict(steps=5000, seed=seed))


def activebox(seed=0, n_owners=4_000_000):
    """The active-box scheme of the paper's rover test (Sec. 6.4) on the
    config-4 bed at a quarter of its size (about 7.5 M spheres in 4 M owners,
    1 m wide): the owners within 0.25 m along x, 0.3 m along y and 0.1 m in
    depth of the rolling cylinder's start are active, the rest dormant
    (fixed, touching only active owners)."""
    s = config4(seed=seed, n_owners=n_owners)
    cyl = s.wall_geom[-1]
    top = s.X[:, 2].max()
    lo = np.array([cyl[0] - 0.25, -0.3, top - 0.1])
    hi = np.array([cyl[0] + 0.25, 0.3, top + 1.0])
    s = active_box(s, lo, hi)
    s.name = "activebox"
    return s


def _qid(n):
    q = np.zeros((n, 4))
    q[:, 0] = 1.0
    return q


def small_spheres(seed, n=200, box=0.05, r=(0.002, 0.003), vel=0.2, walls=True, gravity=(0, 0, -9.81),
                  dt=5e-6, margin=0.0002, mats=None, gap=0.0002, jitter=0.0008):
    """A small random sphere cloud for parity tests (jittered lattice; with
    the default gap and jitter neighbours start overlapping)."""
    rng = np.random.default_rng(seed)
    side = int(math.ceil(n ** (1 / 3)))
    s = 2 * r[1] + gap
    base = lattice((side, side, side), s, -0.5 * (side - 1) * s * np.ones(3), n_take=n)
    rad = rng.uniform(r[0], r[1], size=n)
    jit = rng.uniform(-jitter, jitter, size=(n, 3))
    V = rng.normal(0.0, vel, size=(n, 3))
    Wb = rng.normal(0.0, 20.0, size=(n, 3))
    half = max(box, 0.5 * side * s + 0.004)
    lo, hi = -half * np.ones(3), half * np.ones(3)
    w = box_walls(lo, hi) if walls else concat_walls()
    return assemble(np.full(n, -1), base + jit, _qid(n), V, Wb, [], rad, None, w,
                    mats or materials(), gravity, dt, margin, lo, hi, name=f"small_spheres{seed}")


def small_clumps(seed, n=120, vel=0.2, walls=True, gravity=(0, 0, -9.81), dt=5e-6, margin=0.0002,
                 with_cylinder=False, with_singles=True, spacing=0.0095, jitter=0.0004):
    """Mixed tri-sphere clumps, five-sphere clumps and single spheres (with
    the default spacing neighbouring clumps can start overlapping)."""
    rng = np.random.default_rng(seed)
    side = int(math.ceil(n ** (1 / 3)))
    s = spacing
    base = lattice((side, side, side), s, -0.5 * (side - 1) * s * np.ones(3), n_take=n)
    jit = rng.uniform(-jitter, jitter, size=(n, 3))
    q = random_quaternions(rng, n)
    V = rng.normal(0.0, vel, size=(n, 3))
    Wb = rng.normal(0.0, 20.0, size=(n, 3))
    types = rng.integers(-1 if with_singles else 0, 2, size=n).astype(np.int32)
    q[types < 0] = np.array([1.0, 0, 0, 0])
    half = 0.5 * side * s + 0.006
    lo, hi = -half * np.ones(3), half * np.ones(3)
    ws = [box_walls(lo, hi, moving={0: (0.1, 0.0, 0.0)})] if walls else []
    if with_cylinder:
        ws.append(cylinder((0.0, 0.0, hi[2] - 0.004), (0, 1, 0), 0.01, 0.6 * half, vel=(0.2, 0, 0),
                           omega=(0, 20.0, 0)))
    return assemble(types, base + jit, q, V, Wb,
                    [tri_template(0.003, 0.002), penta_template(0.0025, 0.0025)], 0.0025,
                    [0, 0], concat_walls(*ws), materials(), gravity, dt, margin, lo, hi,
                    name=f"small_clumps{seed}")


# --------------------------------------------------------------------------
# triangle meshes
# --------------------------------------------------------------------------

def add_meshes(sysm, *meshes):
    """Attaches rigid meshes to a system.  Each mesh: dict(tri=[k,3,3]
    vertices in the mesh frame, origin, vel, omega, mat)."""
    tri_mesh, tri_local, org, vel, om, mat = [], [], [], [], [], []
    for g, m in enumerate(meshes):
        tri = snap_pos(np.asarray(m["tri"], dtype=np.float64).reshape(-1, 9))
        tri_local.append(tri)
        tri_mesh.append(np.full(tri.shape[0], g, dtype=np.int32))
        org.append(snap_pos(m.get("origin", (0, 0, 0))))
        vel.append(np.asarray(m.get("vel", (0, 0, 0)), dtype=np.float64))
        om.append(np.asarray(m.get("omega", (0, 0, 0)), dtype=np.float64))
        mat.append(int(m.get("mat", 0)))
    sysm.tri_mesh = np.concatenate(tri_mesh).astype(np.int32)
    sysm.tri_local = np.vstack(tri_local)
    sysm.mesh_origin = np.asarray(org, dtype=np.float64).reshape(-1, 3)
    sysm.mesh_vel = np.asarray(vel, dtype=np.float64).reshape(-1, 3)
    sysm.mesh_omega = np.asarray(om, dtype=np.float64).reshape(-1, 3)
    sysm.mesh_mat = np.asarray(mat, dtype=np.int32)
    return sysm


def quad_grid(p0, e1, e2, n1, n2):
    """A planar parallelogram p0 + a e1 + b e2 (a, b in [0, 1]) split into
    n1 x n2 cells of two triangles each: [2 n1 n2, 3, 3]."""
    p0, e1, e2 = (np.asarray(v, dtype=np.float64) for v in (p0, e1, e2))
    tris = []
    for i in range(n1):
        for j in range(n2):
            a = p0 + e1 * (i / n1) + e2 * (j / n2)
            b = p0 + e1 * ((i + 1) / n1) + e2 * (j / n2)
            c = p0 + e1 * ((i + 1) / n1) + e2 * ((j + 1) / n2)
            d = p0 + e1 * (i / n1) + e2 * ((j + 1) / n2)
            tris.append([a, b, c])
            tris.append([a, c, d])
    return np.asarray(tris)


def bladed_mixer(radius, height, n_blades=4, hub_radius=None, n_r=15, n_z=12, n_theta=48, n_hub_z=15, phase=0.0):
    """A mixer impeller about the z axis in its own frame: n_blades flat
    vertical blades from the hub to 0.9 radius at the angles
    phase + 2 pi k / n_blades, z in [0, height], and a cylindrical hub, all
    triangulated (4 blades with the defaults: 2880 facets)."""
    hub = hub_radius if hub_radius is not None else 0.08 * radius
    parts = []
    for k in range(n_blades):
        th = phase + 2.0 * np.pi * k / n_blades
        d = np.array([np.cos(th), np.sin(th), 0.0])
        parts.append(quad_grid(hub * d, (0.9 * radius - hub) * d, (0, 0, height), n_r, n_z))
    ring = []
    for i in range(n_theta):
        a0, a1 = 2 * np.pi * i / n_theta, 2 * np.pi * (i + 1) / n_theta
        for j in range(n_hub_z):
            z0, z1 = height * j / n_hub_z, height * (j + 1) / n_hub_z
            p = lambda a, z: np.array([hub * np.cos(a), hub * np.sin(a), z])
            ring.append([p(a0, z0), p(a1, z0), p(a1, z1)])
            ring.append([p(a0, z0), p(a1, z1), p(a0, z1)])
    parts.append(np.asarray(ring))
    return np.concatenate(parts)


def small_mixer(seed, n=400, vel=0.1, omega_z=2.0 * np.pi, dt=2e-6, margin=0.0002, r=(0.002, 0.003)):
    """Spheres dropped into a small box chamber (10 x 10 cm) over a rotating
    bladed impeller mesh (radius 4.75 cm), for parity tests."""
    rng = np.random.default_rng(seed)
    R, H = 0.05, 0.03
    side = int(math.ceil((n * 2) ** (1 / 3)))
    s = 2 * r[1] + 0.0006
    pts = []
    z = H + 0.004
    while len(pts) < n:
        for ix in range(-side, side + 1):
            for iy in range(-side, side + 1):
                x, y = ix * s, iy * s
                if x * x + y * y < (R - 2 * r[1]) ** 2 and len(pts) < n:
                    pts.append((x, y, z))
        z += s
    X = np.asarray(pts[:n]) + rng.uniform(-0.0003, 0.0003, size=(n, 3))
    rad = rng.uniform(r[0], r[1], size=n)
    V = rng.normal(0.0, vel, size=(n, 3))
    lo = np.array([-R - 0.004, -R - 0.004, -0.004])
    hi = np.array([R + 0.004, R + 0.004, z + 0.02])
    walls = box_walls(np.array([-R, -R, 0.0]), np.array([R, R, z + 0.02]))
    mats = materials(E=1e8, nu=0.3, cor=0.4, mu=0.5)
    sysm = assemble(np.full(n, -1), X, _qid(n), V, np.zeros((n, 3)), [], rad, None, walls, mats,
                    (0, 0, -9.81), dt, margin, lo, hi, name=f"small_mixer{seed}")
    tri = bladed_mixer(R * 0.95, H, n_r=4, n_z=3, n_theta=12, n_hub_z=3)
    return add_meshes(sysm, dict(tri=tri, origin=(0, 0, 0.0005), omega=(0, 0, omega_z)))


def _blade_clearance(X, radius, height, n_blades, hub, origin, phase):
    """Distance of points X [n,3] to the impeller of bladed_mixer (blades as
    flat rectangles, hub as a cylinder side), for placing spheres clear of it."""
    P = X - np.asarray(origin, dtype=np.float64)[None]
    best = np.full(X.shape[0], np.inf)
    for k in range(n_blades):
        th = phase + 2.0 * np.pi * k / n_blades
        d = np.array([np.cos(th), np.sin(th), 0.0])
        a = np.clip(P @ d, hub, 0.9 * radius)
        z = np.clip(P[:, 2], 0.0, height)
        q = a[:, None] * d[None] + z[:, None] * np.array([0.0, 0.0, 1.0])[None]
        best = np.minimum(best, np.linalg.norm(P - q, axis=1))
    rho = np.hypot(P[:, 0], P[:, 1])
    dz = np.maximum(np.maximum(-P[:, 2], P[:, 2] - height), 0.0)
    best = np.minimum(best, np.hypot(np.abs(rho - hub), dz))
    return best


def set_families(sysm, owner_family=None, pair_off=(), fixed=(), wall_family=None, mesh_family=None):
    """Family tags (the paper's Sec. 2.2.2): a family 0..255 per owner, wall
    and mesh; `pair_off` lists family pairs (a, b) whose contacts are never
    resolved (both orders); `fixed` lists families whose owners stay in
    place (their velocities are zeroed here)."""
    No = sysm.n_owners
    sysm.owner_family = np.asarray(owner_family if owner_family is not None else np.zeros(No), dtype=np.uint8)
    sysm.wall_family = np.asarray(wall_family if wall_family is not None else np.zeros(sysm.n_walls), dtype=np.uint8)
    sysm.mesh_family = np.asarray(mesh_family if mesh_family is not None else np.zeros(sysm.n_mesh), dtype=np.uint8)
    off = np.zeros((256, 256), dtype=np.uint8)
    for a, b in pair_off:
        off[a, b] = off[b, a] = 1
    sysm.fam_pair_off = off.reshape(-1)
    fx = np.zeros(256, dtype=np.uint8)
    fx[list(fixed)] = 1
    sysm.fam_fixed = fx
    still = fx[sysm.owner_family] > 0
    sysm.V = sysm.V.copy()
    sysm.W = sysm.W.copy()
    sysm.V[still] = 0.0
    sysm.W[still] = 0.0
    return sysm


def active_box(sysm, lo, hi, active=0, dormant=1, walls=2, meshes=3):
    """The active-box scheme of the paper's rover test (Sec. 6.4): owners
    whose centre lies outside the box [lo, hi] go to family `dormant`, which
    is fixed and has its contacts with itself, with the walls (family
    `walls`) and with the meshes (family `meshes`) switched off, so the
    dormant owners touch only active ones; owners inside go to family
    `active`."""
    inside = np.all((sysm.X >= np.asarray(lo)) & (sysm.X <= np.asarray(hi)), axis=1)
    fam = np.where(inside, active, dormant).astype(np.uint8)
    return set_families(sysm, fam, pair_off=[(dormant, dormant), (dormant, walls), (dormant, meshes)],
                        fixed=[dormant], wall_family=np.full(sysm.n_walls, walls),
                        mesh_family=np.full(sysm.n_mesh, meshes))


def mixer_bed(seed, n, R, Hb, r, E, cor, dt, margin, omega_z, mesh_res, vel=0.0, name="mixer", packing="cubic",
              gap=0.0002, jitter=0.0001):
    """Spheres r ~ U(r) on a jittered lattice filling, from the floor up, the
    cylinder of radius R inside a 2R x 2R box chamber, around a bladed
    impeller (radius 0.98 R, blade height Hb, turning at omega_z about z):
    lattice sites closer than r_max + 0.3 mm to the impeller are left empty,
    so the blades start inside the bed and sweep it from the first step (the
    blades are turned by 0.3 rad against the lattice rows, so the gaps in
    front of them spread from 0.3 mm to one lattice spacing).  The lattice is
    simple cubic or face-centred cubic with nearest-neighbour distance
    2 r_max + gap, each site jittered by U(-jitter, jitter) per axis."""
    rng = np.random.default_rng(seed)
    s = 2 * r[1] + gap
    if packing == "fcc":
        h = s / np.sqrt(2.0)     # half the cubic cell: the layer spacing and the in-layer grid step
    else:
        h = s
    per = int((2 * R) // h)
    ax = (np.arange(per) - 0.5 * (per - 1)) * h
    # x fastest inside a layer: consecutive ids are neighbours along x, so
    # the bins of a wave of consecutive spheres are consecutive too
    I, J = np.meshgrid(np.arange(per), np.arange(per), indexing="xy")
    XY = np.c_[ax[I.ravel()], ax[J.ravel()]]
    parity = (I.ravel() + J.ravel()) & 1
    inside = (XY ** 2).sum(1) < (R - r[1] - 0.002) ** 2
    Ri = 0.98 * R
    hub = 0.08 * Ri
    origin = (0.0, 0.0, 0.001)
    phase = 0.3
    pts, k = [], 0
    total = 0
    while total < n:
        sel = inside & (parity == (k & 1)) if packing == "fcc" else inside
        layer = XY[sel]
        Xl = np.c_[layer, np.full(layer.shape[0], r[1] + 0.0001 + k * h)]
        keep = _blade_clearance(Xl, Ri, Hb, 4, hub, origin, phase) > r[1] + 0.0003
        pts.append(Xl[keep])
        total += int(keep.sum())
        k += 1
    X = np.vstack(pts)[:n]
    X = X + rng.uniform(-jitter, jitter, size=X.shape)
    rad = rng.uniform(r[0], r[1], size=n)
    V = rng.normal(0.0, vel, size=(n, 3)) if vel > 0 else np.zeros((n, 3))
    top = X[:, 2].max() + 0.02
    lo = np.array([-R - 0.005, -R - 0.005, -0.005])
    hi = np.array([R + 0.005, R + 0.005, top])
    walls = box_walls(np.array([-R, -R, 0.0]), np.array([R, R, top]))
    mats = materials(E=E, nu=0.3, cor=cor, mu=0.5)
    sysm = assemble(np.full(n, -1), X, _qid(n), V, np.zeros((n, 3)), [], rad, None, walls, mats,
                    (0, 0, -9.81), dt, margin, lo, hi, name=name, meta=dict(seed=seed))
    tri = bladed_mixer(Ri, Hb, phase=phase, **mesh_res)
    return add_meshes(sysm, dict(tri=tri, origin=origin, omega=(0, 0, omega_z)))


def small_mixer_bed(seed, n=500, omega_z=20.0 * np.pi, vel=0.05):
    """A small mixer bed for parity tests: 10 x 10 cm chamber, impeller of
    radius 4.9 cm and blade height 2 cm (168 facets) turning at 10 rev/s (tip
    speed 2.8 m/s, as in the full-size mixer),
    r ~ U(2, 3) mm, E = 1e8 Pa, dt = 2e-6 s, margin 0.2 mm."""
    return mixer_bed(seed, n, 0.05, 0.02, (0.002, 0.003), 1e8, 0.4, 2e-6, 0.0002, omega_z,
                     dict(n_r=4, n_z=3, n_theta=12, n_hub_z=3), vel=vel, name=f"small_mixer_bed{seed}")


def mixer(seed=0, n=1_000_000, r=(0.003, 0.0035)):
    """The scaling workload of the paper's Sec. 5 with a synthetic mesh: a
    bladed impeller of 2880 facets (radius 0.49 m, blade height 0.15 m)
    turning at 2 pi rad/s about z in a 1 x 1 m box chamber, inside a dense
    bed of spheres r ~ U(3, 3.5) mm on a face-centred cubic lattice (nearest
    neighbours 7.05 mm apart, jittered by 0.01 mm, so gaps of about 0.02 to
    1.05 mm) filling the
    cylinder of radius 0.5 m from the floor up (about 0.32 m for 1M spheres,
    the paper's 1/3 m; the paper's run is timed in the mixing state after the
    release has settled, which this packed bed stands in for); E = 1e9 Pa,
    nu = 0.3, CoR = 0.2, rho = 2600; dt = 5e-7 s; margin 0.1 r_min."""
    sysm = mixer_bed(seed, n, 0.5, 0.15, r, 1e9, 0.2, 5e-7, 0.1 * r[0], 2.0 * np.pi, {}, name="mixer",
                     packing="fcc", gap=0.00005, jitter=0.00001)
    sysm.meta["steps"] = 5000
    return sysm
