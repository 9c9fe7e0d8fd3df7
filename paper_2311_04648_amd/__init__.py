"""MI355X (gfx950) DEM hot path: thin Python binding over the C ABI in
``include/dem.h``.

Every step of the path runs in the HIP kernels of ``_dem_hip.so``; this
module only marshals arguments.  PyTorch provides the device workspace and the
streams.  The binding fails loudly when the library is not built or no GPU is
visible -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_dem_hip.so")

DEM_OK, DEM_ERR_ARG, DEM_ERR_CAPACITY, DEM_ERR_HIP, DEM_ERR_DIVERGED, DEM_ERR_MISSED, DEM_ERR_STATE = range(7)
MODES = {"every": 0, "fixed": 1, "learned": 2, "adaptive": 3}
MLP_NPARAM = 1313
MLP_NFEAT = 6
_STATUS = {0: "OK", 1: "ARG", 2: "CAPACITY", 3: "HIP", 4: "DIVERGED", 5: "MISSED", 6: "STATE"}


class DemError(RuntimeError):
    def __init__(self, status, msg, required=None):
        super().__init__(f"DEM_ERR_{_STATUS.get(status, status)}: {msg}")
        self.status = status
        self.required = required


class Params(C.Structure):
    _fields_ = [("gravity", C.c_double * 3), ("dt", C.c_double), ("margin", C.c_double),
                ("v_error_out", C.c_double), ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
                ("cd_mode", C.c_int32), ("cd_interval", C.c_int32), ("cd_latency", C.c_int32),
                ("judge", C.c_int32), ("repair", C.c_int32), ("cd_interval_max", C.c_int32),
                ("timing", C.c_int32), ("mlp_safety", C.c_double), ("bin_sort", C.c_int32),
                ("dyn_path", C.c_int32), ("no_pair_skip", C.c_int32)]


class Materials(C.Structure):
    _fields_ = [("n", C.c_int32), ("E", C.c_void_p), ("nu", C.c_void_p), ("cor", C.c_void_p),
                ("mu", C.c_void_p), ("crr", C.c_void_p)]


class Templates(C.Structure):
    _fields_ = [("n", C.c_int32), ("sph_begin", C.c_void_p), ("sph_pos", C.c_void_p)]


class Walls(C.Structure):
    _fields_ = [("n", C.c_int32), ("type", C.c_void_p), ("geom", C.c_void_p), ("vel", C.c_void_p),
                ("omega", C.c_void_p), ("mat", C.c_void_p)]


class Meshes(C.Structure):
    _fields_ = [("n_mesh", C.c_int32), ("n_tri", C.c_int64), ("tri_mesh", C.c_void_p), ("tri_local", C.c_void_p),
                ("origin", C.c_void_p), ("vel", C.c_void_p), ("omega", C.c_void_p), ("mat", C.c_void_p)]


class Families(C.Structure):
    _fields_ = [("owner_family", C.c_void_p), ("wall_family", C.c_void_p), ("mesh_family", C.c_void_p),
                ("pair_off", C.c_void_p), ("fixed", C.c_void_p)]


class Bodies(C.Structure):
    _fields_ = [("n_owners", C.c_int64), ("n_spheres", C.c_int64), ("own_sph0", C.c_void_p),
                ("own_tmpl", C.c_void_p), ("own_mass", C.c_void_p), ("own_moi", C.c_void_p),
                ("sph_comp", C.c_void_p), ("sph_rad", C.c_void_p), ("sph_mat", C.c_void_p)]


class StepStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("step", C.c_int64), ("cds", C.c_int64), ("swaps", C.c_int64),
                ("misses", C.c_int64), ("repairs", C.c_int64), ("n_contacts", C.c_int64),
                ("required_capacity", C.c_int64), ("max_speed", C.c_double), ("ms", C.c_double),
                ("mean_interval", C.c_double), ("stage_ms", C.c_double * 5), ("stage_n", C.c_int64 * 5),
                ("mean_contacts", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["stage_ms"] = list(self.stage_ms)
        d["stage_n"] = list(self.stage_n)
        return d


_lib = None


def lib():
    """Loads the HIP library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, d, f = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_float
        sig = {
            "dem_create": [vp, vp, vp, vp, vp, vp],
            "dem_set_meshes": [vp, vp],
            "dem_set_families": [vp, vp, vp],
            "dem_workspace_size": [vp, i64, vp],
            "dem_bind": [vp, vp, i64, i64],
            "dem_set_state": [vp, vp, vp, vp, vp, i64, vp],
            "dem_get_state": [vp, vp, vp, vp, vp, vp, vp],
            "dem_bin": [vp, vp, vp, vp],
            "dem_detect_contacts": [vp, d, vp, vp],
            "dem_forces": [vp, vp],
            "dem_get_forces": [vp, vp, vp, vp, i64, vp],
            "dem_step": [vp, i64, vp, vp, vp],
            "dem_get_contacts": [vp, vp, vp, i64, vp, vp],
            "dem_set_contacts": [vp, vp, vp, i64, vp],
            "dem_count_missing": [vp, vp, vp],
            "dem_mlp_set": [vp, vp],
            "dem_features": [vp, vp, i64, vp, vp],
            "dem_mlp_forward": [vp, vp, vp, i64, vp],
            "dem_mlp_backward": [vp, vp, vp, i64, f, vp, vp, vp, i64, vp],
            "dem_mlp_backward_noalloc": [vp, vp, vp, i64, f, vp, vp, vp],
            "dem_mlp_adam": [vp, vp, vp, vp, i64, f, f, f, f, vp],
            "dem_snapshot": [vp, vp],
            "dem_feature_cells": [vp, vp, i64, vp, vp, vp],
            "dem_label_begin": [vp, vp, vp],
            "dem_label_update": [vp, C.c_uint32, vp, vp],
            "dem_info": [vp, vp, i64],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = i32
        L.dem_mlp_backward_work_bytes.argtypes = [i64]
        L.dem_mlp_backward_work_bytes.restype = i64
        L.dem_last_error.argtypes = [vp]
        L.dem_last_error.restype = C.c_char_p
        L.dem_destroy.argtypes = [vp]
        L.dem_destroy.restype = None
        _lib = L
    return _lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the DEM library runs on an MI355X only")
    return torch


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream))


def _p(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class DemContext:
    """One DEM problem bound to caller-owned device memory (a torch tensor)."""

    def __init__(self, system, mode="every", k=10, lam=5, judge=False, repair=True, capacity=None,
                 margin=None, v_error_out=0.0, k_max=None, device="cuda:0", timing=False, mlp_safety=1.0,
                 bin_sort=0, dyn_path=0, pair_skip=True):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.sys = system
        L = lib()
        s = system
        self._keep = []

        def keep(a, dt):
            a = _c(a, dt)
            self._keep.append(a)
            return a.ctypes.data

        P = Params()
        for i in range(3):
            P.gravity[i] = float(s.gravity[i])
            P.domain_lo[i] = float(s.domain_lo[i])
            P.domain_hi[i] = float(s.domain_hi[i])
        P.dt = float(s.dt)
        P.margin = float(s.margin if margin is None else margin)
        P.v_error_out = float(v_error_out)
        P.cd_mode = MODES[mode]
        P.cd_interval = int(k)
        P.cd_latency = int(lam)
        P.judge = int(bool(judge))
        P.repair = int(bool(repair))
        P.cd_interval_max = int(k_max or 16 * max(int(k), 1))
        P.timing = int(timing) if not isinstance(timing, bool) else int(timing)
        P.mlp_safety = float(mlp_safety)
        P.bin_sort = int(bin_sort)
        P.dyn_path = int(dyn_path)
        P.no_pair_skip = 0 if pair_skip else 1
        self.params = P
        Mt = Materials(int(np.asarray(s.mat_E).shape[0]), keep(s.mat_E, np.float64), keep(s.mat_nu, np.float64),
                       keep(s.mat_cor, np.float64), keep(s.mat_mu, np.float64), keep(s.mat_crr, np.float64))
        T = Templates(int(s.tmpl_sph0.shape[0] - 1), keep(s.tmpl_sph0, np.int32), keep(s.tmpl_local, np.float64))
        Wl = Walls(int(s.wall_type.shape[0]), keep(s.wall_type, np.int32), keep(s.wall_geom, np.float64),
                   keep(s.wall_vel, np.float64), keep(s.wall_omega, np.float64), keep(s.wall_mat, np.int32))
        B = Bodies(int(s.own_tmpl.shape[0]), int(s.sph_rad.shape[0]), keep(s.own_sph0, np.int32),
                   keep(s.own_tmpl, np.int32), keep(s.own_mass, np.float64), keep(s.own_moi, np.float64),
                   keep(s.sph_comp, np.int32), keep(s.sph_rad, np.float64), keep(s.sph_mat, np.int32))
        ctx = C.c_void_p()
        st = L.dem_create(C.byref(P), C.byref(Mt), C.byref(T), C.byref(Wl), C.byref(B), C.byref(ctx))
        self.ctx = ctx
        if st != DEM_OK:
            msg = L.dem_last_error(ctx).decode() if ctx else "dem_create failed"
            if ctx:
                L.dem_destroy(ctx)
            self.ctx = None
            raise DemError(st, msg)
        n_mesh = int(getattr(s, "n_mesh", 0))
        if n_mesh > 0:
            Ms = Meshes(n_mesh, int(s.n_tri), keep(s.tri_mesh, np.int32), keep(s.tri_local, np.float64),
                        keep(s.mesh_origin, np.float64), keep(s.mesh_vel, np.float64),
                        keep(s.mesh_omega, np.float64), keep(s.mesh_mat, np.int32))
            st = L.dem_set_meshes(ctx, C.byref(Ms))
            if st != DEM_OK:
                msg = L.dem_last_error(ctx).decode()
                L.dem_destroy(ctx)
                self.ctx = None
                raise DemError(st, msg)
        self._keep.clear()
        self.No = int(s.own_tmpl.shape[0])
        self.Ns = int(s.sph_rad.shape[0])
        self.capacity = int(capacity or max(64, 12 * self.Ns))
        self.bind(self.capacity)
        if np.asarray(getattr(s, "owner_family", np.zeros(0))).size:
            self.set_families(s.owner_family, s.wall_family, s.mesh_family, s.fam_pair_off, s.fam_fixed)

    # ------------------------------------------------------------------ core
    def _check(self, st, required=None):
        if st != DEM_OK:
            raise DemError(st, lib().dem_last_error(self.ctx).decode(), required)

    def bind(self, capacity):
        L = lib()
        nbytes = C.c_int64()
        self._check(L.dem_workspace_size(self.ctx, int(capacity), C.byref(nbytes)))
        self.workspace = None
        self.workspace = self.torch.empty(int(nbytes.value), dtype=self.torch.uint8, device=self.device)
        self.capacity = int(capacity)
        self._check(L.dem_bind(self.ctx, C.c_void_p(self.workspace.data_ptr()), int(nbytes.value), int(capacity)))
        self.workspace_bytes = int(nbytes.value)

    def close(self):
        if getattr(self, "ctx", None):
            lib().dem_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_families(self, owner_family=None, wall_family=None, mesh_family=None, pair_off=None, fixed=None,
                     stream=None):
        """Family tags: owner_family [No], wall_family [W], mesh_family [M],
        pair_off [256*256] (1 = no contact between the two families), fixed
        [256]; None = all 0.  With a state set, the set is rebuilt at once."""
        keep = []

        def u8(a, n):
            if a is None or np.asarray(a).size == 0:
                return None
            a = np.ascontiguousarray(a, dtype=np.uint8).reshape(-1)
            if a.size != n:
                raise ValueError(f"family array of {a.size} entries, expected {n}")
            keep.append(a)
            return a.ctypes.data

        s = self.sys
        F = Families(u8(owner_family, self.No), u8(wall_family, int(s.wall_type.shape[0])),
                     u8(mesh_family, int(getattr(s, "n_mesh", 0))), u8(pair_off, 65536), u8(fixed, 256))
        self._check(lib().dem_set_families(self.ctx, C.byref(F), _stream_ptr(stream)))

    def set_state(self, X=None, q=None, V=None, W=None, step=0, stream=None):
        s = self.sys
        X = _c(s.X if X is None else X, np.float64)
        q = _c(s.q if q is None else q, np.float64)
        V = _c(s.V if V is None else V, np.float32)
        W = _c(s.W if W is None else W, np.float32)
        self._check(lib().dem_set_state(self.ctx, _p(X), _p(q), _p(V), _p(W), int(step), _stream_ptr(stream)))

    def get_state(self, stream=None):
        X = np.zeros((self.No, 3))
        q = np.zeros((self.No, 4))
        V = np.zeros((self.No, 3), dtype=np.float32)
        W = np.zeros((self.No, 3), dtype=np.float32)
        step = C.c_int64()
        self._check(lib().dem_get_state(self.ctx, _p(X), _p(q), _p(V), _p(W), C.byref(step), _stream_ptr(stream)))
        return dict(X=X, q=q, V=V, W=W, step=int(step.value))

    def bin(self, stream=None, read=True):
        keys = np.zeros(self.Ns, dtype=np.uint32) if read else None
        ids = np.zeros(self.Ns, dtype=np.uint32) if read else None
        self._check(lib().dem_bin(self.ctx, _stream_ptr(stream), _p(keys), _p(ids)))
        return keys, ids

    def detect_contacts(self, margin=0.0, stream=None, sync=True):
        n = C.c_int64()
        st = lib().dem_detect_contacts(self.ctx, float(margin), _stream_ptr(stream), C.byref(n) if sync else None)
        self._check(st, int(n.value) if st == DEM_ERR_CAPACITY else None)
        return int(n.value) if sync else None

    def forces(self, stream=None):
        self._check(lib().dem_forces(self.ctx, _stream_ptr(stream)))

    def get_forces(self, n_contacts=None, stream=None):
        Fo = np.zeros((self.No, 3), dtype=np.float32)
        To = np.zeros((self.No, 3), dtype=np.float32)
        n = self.capacity if n_contacts is None else int(n_contacts)
        Fc = np.zeros((max(n, 1), 3), dtype=np.float32)
        self._check(lib().dem_get_forces(self.ctx, _p(Fo), _p(To), _p(Fc), n, _stream_ptr(stream)))
        return Fo, To, Fc[:n]

    def get_contacts(self, stream=None):
        n = C.c_int64()
        st = lib().dem_get_contacts(self.ctx, None, None, 0, C.byref(n), _stream_ptr(stream))
        if st not in (DEM_OK, DEM_ERR_CAPACITY) or n.value > self.capacity:
            self._check(st if st != DEM_OK else DEM_ERR_CAPACITY)
        cap = int(n.value)
        keys = np.zeros(max(cap, 1), dtype=np.uint64)
        hist = np.zeros((max(cap, 1), 4), dtype=np.float32)
        self._check(lib().dem_get_contacts(self.ctx, _p(keys), _p(hist), cap, C.byref(n), _stream_ptr(stream)))
        n = int(n.value)
        return keys[:n], hist[:n]

    def set_contacts(self, keys, hist=None, stream=None):
        """hist: [n,4] (displacement xyz, age) or [n,3] (age 0)."""
        keys = _c(keys, np.uint64)
        h = None
        if hist is not None:
            hh = _c(hist, np.float32).reshape(keys.shape[0], -1)
            h = np.zeros((keys.shape[0], 4), dtype=np.float32)
            h[:, : hh.shape[1]] = hh
        self._check(lib().dem_set_contacts(self.ctx, _p(keys), _p(h), int(keys.shape[0]), _stream_ptr(stream)))

    def count_missing(self, stream=None):
        n = C.c_int64()
        self._check(lib().dem_count_missing(self.ctx, _stream_ptr(stream), C.byref(n)))
        return int(n.value)

    def step(self, n_steps, dyn=None, kin=None):
        stats = StepStats()
        st = lib().dem_step(self.ctx, int(n_steps), _stream_ptr(dyn), _stream_ptr(kin), C.byref(stats))
        self._check(st, stats.required_capacity if st == DEM_ERR_CAPACITY else None)
        return stats.as_dict()

    # --------------------------------------------------------- learned part
    def mlp_set(self, params):
        p = None if params is None else _c(params, np.float32)
        if p is not None and p.size != MLP_NPARAM:
            raise ValueError("MLP needs 1313 parameters")
        self._check(lib().dem_mlp_set(self.ctx, _p(p)))

    def snapshot(self, stream=None):
        self._check(lib().dem_snapshot(self.ctx, _stream_ptr(stream)))

    def info(self):
        v = np.zeros(8, dtype=np.int64)
        self._check(lib().dem_info(self.ctx, _p(v), 8))
        return dict(nbins=int(v[0]), ncells=int(v[1]), nx=int(v[2]), ny=int(v[3]), nz=int(v[4]),
                    sort_bits=int(v[5]), capacity=int(v[6]), step=int(v[7]))

    def features(self, stream=None):
        """Features of occupied cells (torch float32 [n,6] on the device),
        the cell id of each row and the cell of each owner."""
        torch = self.torch
        ncell_total = self.info()["ncells"]
        out = torch.empty((max(ncell_total, 1), MLP_NFEAT), dtype=torch.float32, device=self.device)
        n = C.c_int64()
        self._check(lib().dem_features(self.ctx, C.c_void_p(out.data_ptr()), ncell_total, C.byref(n),
                                       _stream_ptr(stream)))
        n = int(n.value)
        ids = np.zeros(max(n, 1), dtype=np.uint32)
        own = np.zeros(self.No, dtype=np.uint32)
        tot = C.c_int64()
        self._check(lib().dem_feature_cells(self.ctx, _p(ids), n, _p(own), C.byref(tot), _stream_ptr(stream)))
        return out[:n], ids[:n], own

    def label_begin(self, stream=None):
        n = C.c_int64()
        self._check(lib().dem_label_begin(self.ctx, _stream_ptr(stream), C.byref(n)))
        return int(n.value)

    def label_update(self, t, first_miss, stream=None):
        self._check(lib().dem_label_update(self.ctx, int(t), C.c_void_p(first_miss.data_ptr()),
                                           _stream_ptr(stream)))


# ---------------------------------------------------------------------------
# stand-alone MLP kernels on torch device tensors
# ---------------------------------------------------------------------------
def _dptr(t):
    return C.c_void_p(t.data_ptr())


def mlp_forward(params, X, stream=None):
    torch = _torch()
    n = int(X.shape[0])
    Y = torch.empty(n, dtype=torch.float32, device=X.device)
    st = lib().dem_mlp_forward(_dptr(params), _dptr(X), _dptr(Y), n, _stream_ptr(stream))
    if st != DEM_OK:
        raise DemError(st, "dem_mlp_forward failed")
    return Y


def mlp_backward(params, X, T, tau, stream=None):
    torch = _torch()
    n = int(X.shape[0])
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    wb = int(lib().dem_mlp_backward_work_bytes(n))
    work = torch.empty(wb // 4 + 1, dtype=torch.float32, device=X.device)
    st = lib().dem_mlp_backward(_dptr(params), _dptr(X), _dptr(T), n, float(tau), _dptr(grad), _dptr(loss),
                                _dptr(work), wb, _stream_ptr(stream))
    if st != DEM_OK:
        raise DemError(st, "dem_mlp_backward failed")
    return grad, loss


MLP_NOALLOC_MAX = 49152   # DEM_MLP_NOALLOC_MAX


def mlp_backward_noalloc(params, X, T, tau, grad, loss, stream=None):
    """dem_mlp_backward_noalloc: the gradient into the caller's `grad`
    [1313] and `loss` [1] (float32 device tensors); no device memory is
    allocated by the library or here (its scratch is a fixed device array,
    shared by every call on the GPU)."""
    n = int(X.shape[0])
    st = lib().dem_mlp_backward_noalloc(_dptr(params), _dptr(X), _dptr(T), n, float(tau), _dptr(grad),
                                        _dptr(loss), _stream_ptr(stream))
    if st != DEM_OK:
        raise DemError(st, lib().dem_last_error(None).decode())
    return grad, loss


def mlp_adam(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    st = lib().dem_mlp_adam(_dptr(params), _dptr(grad), _dptr(m), _dptr(v), int(t), float(lr), float(beta1),
                            float(beta2), float(eps), _stream_ptr(stream))
    if st != DEM_OK:
        raise DemError(st, "dem_mlp_adam failed")
