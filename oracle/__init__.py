"""FP64 CPU oracle of the DEM hot path (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: the C part
(``dem_oracle.c``) is compiled on its own with gcc, and the MLP part
(``mlp.py``) is plain numpy in float64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dem_oracle.c")
# DEM_ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (any finding aborts); the process must then be
# started with the AddressSanitizer runtime preloaded
SANITIZE = os.environ.get("DEM_ORACLE_SANITIZE", "") == "1"
LIB = os.path.join(HERE, "_dem_oracle_san.so" if SANITIZE else "_dem_oracle.so")


def build(force=False):
    """Compile the C oracle with strict IEEE double arithmetic."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        flags = ["-O2"]
        if SANITIZE:
            flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"]
        subprocess.check_call(["gcc", *flags, "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class OrcSys(C.Structure):
    _fields_ = [
        ("n_owners", C.c_int64), ("n_spheres", C.c_int64),
        ("own_sph0", C.c_void_p), ("own_mass", C.c_void_p), ("own_moi", C.c_void_p),
        ("sph_owner", C.c_void_p), ("sph_local", C.c_void_p), ("sph_rad", C.c_void_p),
        ("sph_mat", C.c_void_p),
        ("n_walls", C.c_int64), ("wall_type", C.c_void_p), ("wall_geom", C.c_void_p),
        ("wall_vel", C.c_void_p), ("wall_omega", C.c_void_p), ("wall_mat", C.c_void_p),
        ("n_mat", C.c_int64), ("mat_E", C.c_void_p), ("mat_nu", C.c_void_p),
        ("mat_cor", C.c_void_p), ("mat_mu", C.c_void_p), ("mat_crr", C.c_void_p),
        ("gravity", C.c_double * 3), ("h", C.c_double),
        ("n_mesh", C.c_int64), ("n_tri", C.c_int64), ("tri_mesh", C.c_void_p), ("tri_local", C.c_void_p),
        ("mesh_origin", C.c_void_p), ("mesh_vel", C.c_void_p), ("mesh_omega", C.c_void_p),
        ("mesh_mat", C.c_void_p),
        ("owner_family", C.c_void_p), ("wall_family", C.c_void_p), ("mesh_family", C.c_void_p),
        ("pair_off", C.c_void_p), ("fixed", C.c_void_p),
    ]


class OrcStats(C.Structure):
    _fields_ = [("cds", C.c_int64), ("swaps", C.c_int64), ("misses", C.c_int64),
                ("repairs", C.c_int64), ("max_acs", C.c_int64), ("sum_acs", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        vp, i64, d = C.c_void_p, C.c_int64, C.c_double
        _lib.orc_sphere_centres.argtypes = [vp, vp, vp, vp]
        _lib.orc_wall_positions.argtypes = [vp, i64, vp]
        _lib.orc_detect_brute.argtypes = [vp, vp, vp, d, vp, i64]
        _lib.orc_detect_brute.restype = i64
        _lib.orc_detect_binned.argtypes = [vp, vp, vp, d, vp, i64]
        _lib.orc_detect_binned.restype = i64
        _lib.orc_detect_row.argtypes = [vp, vp, vp, d, i64, vp, i64]
        _lib.orc_detect_row.restype = i64
        _lib.orc_count_missing.argtypes = [vp, vp, vp, vp, i64, vp, i64]
        _lib.orc_count_missing.restype = i64
        _lib.orc_remap.argtypes = [vp, vp, i64, vp, vp, i64]
        _lib.orc_forces.argtypes = [vp, vp, vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_integrate.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        _lib.orc_run.argtypes = [vp, vp, vp, vp, vp, vp, i64, C.c_int, i64, i64, d, C.c_int,
                                 vp, vp, vp, i64, vp]
        _lib.orc_run.restype = C.c_int
        _lib.orc_tri_closest.argtypes = [vp, vp, vp, vp, vp]
        _lib.orc_mesh_pose.argtypes = [vp, i64, i64, vp, vp]
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def tri_closest(a, b, c, p):
    """Closest point of triangle (a, b, c) to p (FP64)."""
    a, b, c, p = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, p))
    q = np.zeros(3)
    lib().orc_tri_closest(_p(a), _p(b), _p(c), _p(p), _p(q))
    return q


def _hist4(hist, n):
    """Contact history as [n,4] float64 (tangential displacement xyz, contact
    age); a [n,3] input gets age 0."""
    out = np.zeros((n, 4))
    if n:
        h = np.asarray(hist, dtype=np.float64).reshape(n, -1)
        out[:, : h.shape[1]] = h
    return np.ascontiguousarray(out)


class Oracle:
    """Holds one system's constant inputs and runs the oracle on states."""

    def __init__(self, sysm):
        self.sys = sysm
        keep = {}

        def arr(name, dt):
            a = np.ascontiguousarray(getattr(sysm, name), dtype=dt)
            keep[name] = a
            return a.ctypes.data

        def arr_u8(a):
            a = np.ascontiguousarray(a, dtype=np.uint8)
            keep[id(a)] = a
            return a.ctypes.data

        s = OrcSys()
        s.n_owners = sysm.n_owners
        s.n_spheres = sysm.n_spheres
        s.own_sph0 = arr("own_sph0", np.int32)
        s.own_mass = arr("own_mass", np.float64)
        s.own_moi = arr("own_moi", np.float64)
        s.sph_owner = arr("sph_owner", np.int32)
        s.sph_local = arr("sph_local", np.float64)
        s.sph_rad = arr("sph_rad", np.float64)
        s.sph_mat = arr("sph_mat", np.int32)
        s.n_walls = sysm.n_walls
        s.wall_type = arr("wall_type", np.int32)
        s.wall_geom = arr("wall_geom", np.float64)
        s.wall_vel = arr("wall_vel", np.float64)
        s.wall_omega = arr("wall_omega", np.float64)
        s.wall_mat = arr("wall_mat", np.int32)
        s.n_mat = int(np.asarray(sysm.mat_E).shape[0])
        s.mat_E = arr("mat_E", np.float64)
        s.mat_nu = arr("mat_nu", np.float64)
        s.mat_cor = arr("mat_cor", np.float64)
        s.mat_mu = arr("mat_mu", np.float64)
        s.mat_crr = arr("mat_crr", np.float64)
        for k in range(3):
            s.gravity[k] = float(sysm.gravity[k])
        s.h = float(sysm.dt)
        s.n_tri = sysm.n_tri
        s.n_mesh = sysm.n_mesh
        s.tri_mesh = arr("tri_mesh", np.int32)
        s.tri_local = arr("tri_local", np.float64)
        s.mesh_origin = arr("mesh_origin", np.float64)
        s.mesh_vel = arr("mesh_vel", np.float64)
        s.mesh_omega = arr("mesh_omega", np.float64)
        s.mesh_mat = arr("mesh_mat", np.int32)
        # family tags: an empty array means the default (NULL)
        for name in ("owner_family", "wall_family", "mesh_family", "pair_off", "fixed"):
            a = np.asarray(getattr(sysm, "fam_" + name if name in ("pair_off", "fixed") else name,
                                   np.zeros(0)), dtype=np.uint8)
            setattr(s, name, arr_u8(a) if a.size else None)
        self._keep = keep
        self._s = s
        self.ps = C.addressof(s)

    # -------------------------------------------------------------- helpers
    def state(self, st=None):
        st = st if st is not None else self.sys.copy_state()
        return {k: np.ascontiguousarray(st[k], dtype=np.float64).copy() for k in ("X", "q", "V", "W")}

    def sphere_centres(self, st):
        xs = np.zeros((self.sys.n_spheres, 3))
        lib().orc_sphere_centres(self.ps, _p(st["X"]), _p(st["q"]), _p(xs))
        return xs

    def _geom(self, step):
        """Prescribed-motion geometry at a step: wall reference points
        (3 per wall) followed by the world vertices of every facet (9)."""
        wp = np.zeros(3 * self.sys.n_walls + 9 * self.sys.n_tri + 1)
        lib().orc_wall_positions(self.ps, int(step), _p(wp))
        return wp

    def wall_positions(self, step):
        return self._geom(step)[: 3 * self.sys.n_walls].reshape(-1, 3)

    def facet_positions(self, step):
        """World vertices [T, 3, 3] of every facet at a step."""
        W = self.sys.n_walls
        return self._geom(step)[3 * W: 3 * W + 9 * self.sys.n_tri].reshape(-1, 3, 3)

    def mesh_pose(self, g, step):
        p, R = np.zeros(3), np.zeros(9)
        lib().orc_mesh_pose(self.ps, int(g), int(step), _p(p), _p(R))
        return p, R.reshape(3, 3)

    def detect(self, st, margin, step=0, brute=False, cap=None):
        xs = self.sphere_centres(st)
        wp = self._geom(step)
        cap = cap or max(64, 16 * self.sys.n_spheres)
        while True:
            keys = np.zeros(cap, dtype=np.uint64)
            fn = lib().orc_detect_brute if brute else lib().orc_detect_binned
            n = fn(self.ps, _p(xs), _p(wp), float(margin), _p(keys), cap)
            if n >= 0:
                return keys[:n].copy()
            cap = -n

    def detect_rows(self, st, margin, spheres, step=0):
        """Rows of the given spheres by brute force (for sampled checks of
        inputs too large for a full detection)."""
        xs = self.sphere_centres(st)
        wp = self._geom(step)
        out = []
        buf = np.zeros(4096, dtype=np.uint64)
        for i in spheres:
            n = lib().orc_detect_row(self.ps, _p(xs), _p(wp), float(margin), int(i), _p(buf), buf.size)
            out.append(buf[:n].copy())
        return out

    def forces(self, st, keys, hist, step=0):
        n = int(keys.shape[0])
        No, W = self.sys.n_owners, self.sys.n_walls
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        hist = _hist4(hist, n)
        out = dict(Fc=np.zeros((n, 3)), TA=np.zeros((n, 3)), TB=np.zeros((n, 3)),
                   Fo=np.zeros((No, 3)), To=np.zeros((No, 3)), Fw=np.zeros((max(W, 1), 3)),
                   touch=np.zeros(n, dtype=np.int32), scale=np.zeros(n))
        lib().orc_forces(self.ps, _p(st["X"]), _p(st["q"]), _p(st["V"]), _p(st["W"]), int(step),
                         _p(keys), n, _p(hist), _p(out["Fc"]), _p(out["TA"]), _p(out["TB"]),
                         _p(out["Fo"]), _p(out["To"]), _p(out["Fw"]), _p(out["touch"]), _p(out["scale"]))
        out["Fw"] = out["Fw"][:W]
        out["hist"] = hist
        return out

    def integrate(self, st, Fo, To):
        lib().orc_integrate(self.ps, _p(st["X"]), _p(st["q"]), _p(st["V"]), _p(st["W"]),
                            _p(np.ascontiguousarray(Fo, dtype=np.float64)),
                            _p(np.ascontiguousarray(To, dtype=np.float64)))
        return st

    def remap(self, old_keys, old_hist, new_keys):
        new_hist = np.zeros((new_keys.shape[0], 4))
        lib().orc_remap(_p(np.ascontiguousarray(old_keys, dtype=np.uint64)),
                        _p(_hist4(old_hist, old_keys.shape[0])), int(old_keys.shape[0]),
                        _p(np.ascontiguousarray(new_keys, dtype=np.uint64)), _p(new_hist),
                        int(new_keys.shape[0]))
        return new_hist

    def count_missing(self, st, acs, step=0):
        xs = self.sphere_centres(st)
        wp = self._geom(step)
        cap = max(64, 16 * self.sys.n_spheres)
        tmp = np.zeros(cap, dtype=np.uint64)
        acs = np.ascontiguousarray(acs, dtype=np.uint64)
        return int(lib().orc_count_missing(self.ps, _p(xs), _p(wp), _p(acs), int(acs.shape[0]),
                                           _p(tmp), cap))

    def run(self, st, n_steps, mode="every", k=10, lam=5, margin=None, judge=False, step=0,
            acs=None, cap=None):
        """Runs the schedule of Sec. 2.1 (see orc_run).  Returns (state, acs, stats).
        Without `cap` the contact buffers hold four times the set the run
        starts from, and a run that outgrows them is repeated from the same
        inputs with twice the room."""
        margin = self.sys.margin if margin is None else margin
        if cap is None:
            n0 = self.detect(st, margin if mode != "every" else 0.0, step=step).size
            n0 = max(n0, 0 if acs is None else acs[0].shape[0])
            cap = 4 * n0 + 4096
            st0 = {k: v.copy() for k, v in st.items()}
            while True:
                try:
                    return self.run(st, n_steps, mode=mode, k=k, lam=lam, margin=margin, judge=judge, step=step,
                                    acs=acs, cap=cap)
                except RuntimeError:
                    for key, v in st0.items():
                        st[key][...] = v
                    cap *= 2
        keys = np.zeros(cap, dtype=np.uint64)
        hist = np.zeros((cap, 4))
        n_acs = np.zeros(1, dtype=np.int64)
        if acs is not None:
            keys[: acs[0].shape[0]] = acs[0]
            hist[: acs[0].shape[0]] = _hist4(acs[1], acs[0].shape[0])
            n_acs[0] = acs[0].shape[0]
        stepv = np.array([step], dtype=np.int64)
        stats = OrcStats()
        rc = lib().orc_run(self.ps, _p(st["X"]), _p(st["q"]), _p(st["V"]), _p(st["W"]), _p(stepv),
                           int(n_steps), 0 if mode == "every" else 1, int(k), int(lam), float(margin),
                           int(bool(judge)), _p(keys), _p(hist), _p(n_acs), cap, C.addressof(stats))
        if rc != 0:
            raise RuntimeError("oracle contact capacity exceeded")
        n = int(n_acs[0])
        return st, (keys[:n].copy(), hist[:n].copy()), stats.as_dict(), int(stepv[0])
