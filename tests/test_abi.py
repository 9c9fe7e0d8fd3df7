"""CPU checks of the C ABI: the library builds, loads, and exports every
entry point that include/dem.h declares; argument validation that runs on
the host needs no GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2311_04648_amd as dem
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ensure_built():
    if not os.path.exists(dem.LIB_PATH):
        from paper_2311_04648_amd import build
        build.build()


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dem.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    _ensure_built()
    L = C.CDLL(dem.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 25
    for name in syms:
        assert hasattr(L, name), name


def test_header_declares_every_exported_symbol():
    _ensure_built()
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", dem.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (dem_[a-z0-9_]+)", out)))
    assert exported == declared_symbols()


def _create(sysm, **kw):
    """dem_create only (host work, no device calls)."""
    L = dem.lib()
    P = dem.Params()
    for i in range(3):
        P.gravity[i] = sysm.gravity[i]
        P.domain_lo[i] = sysm.domain_lo[i]
        P.domain_hi[i] = sysm.domain_hi[i]
    P.dt = kw.get("dt", sysm.dt)
    P.margin = sysm.margin
    P.cd_mode = kw.get("mode", 1)
    P.cd_interval = kw.get("k", 10)
    P.cd_latency = kw.get("lam", 5)
    P.dyn_path = kw.get("dyn_path", 0)
    P.bin_sort = kw.get("bin_sort", 0)
    keep = []

    def k(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data

    Mt = dem.Materials(1, k(sysm.mat_E, np.float64), k(sysm.mat_nu, np.float64), k(sysm.mat_cor, np.float64),
                       k(sysm.mat_mu, np.float64), k(sysm.mat_crr, np.float64))
    T = dem.Templates(int(sysm.tmpl_sph0.shape[0] - 1), k(sysm.tmpl_sph0, np.int32), k(sysm.tmpl_local, np.float64))
    Wl = dem.Walls(int(sysm.n_walls), k(sysm.wall_type, np.int32), k(sysm.wall_geom, np.float64),
                   k(sysm.wall_vel, np.float64), k(sysm.wall_omega, np.float64), k(sysm.wall_mat, np.int32))
    sph_rad = kw.get("sph_rad", sysm.sph_rad)
    B = dem.Bodies(sysm.n_owners, sysm.n_spheres, k(sysm.own_sph0, np.int32), k(sysm.own_tmpl, np.int32),
                   k(sysm.own_mass, np.float64), k(sysm.own_moi, np.float64), k(sysm.sph_comp, np.int32),
                   k(sph_rad, np.float64), k(sysm.sph_mat, np.int32))
    ctx = C.c_void_p()
    st = L.dem_create(C.byref(P), C.byref(Mt), C.byref(T), C.byref(Wl), C.byref(B), C.byref(ctx))
    msg = L.dem_last_error(ctx).decode() if ctx else ""
    return st, ctx, msg


def test_create_and_workspace_size_on_host():
    _ensure_built()
    s = W.small_clumps(0, n=50, with_cylinder=True)
    st, ctx, msg = _create(s)
    assert st == dem.DEM_OK, msg
    nb = C.c_int64()
    assert dem.lib().dem_workspace_size(ctx, 1000, C.byref(nb)) == dem.DEM_OK
    nb2 = C.c_int64()
    assert dem.lib().dem_workspace_size(ctx, 2000, C.byref(nb2)) == dem.DEM_OK
    assert nb2.value > nb.value > 0
    v = np.zeros(8, dtype=np.int64)
    assert dem.lib().dem_info(ctx, v.ctypes.data, 8) == dem.DEM_OK
    assert v[0] == v[2] * v[3] * v[4] and v[1] > 0
    dem.lib().dem_destroy(ctx)


@pytest.mark.parametrize("bad", ["dt", "radius", "latency", "mode", "adaptive_latency", "dyn_path", "bin_sort"])
def test_create_rejects_bad_arguments(bad):
    _ensure_built()
    s = W.small_spheres(0, n=20)
    kw = {}
    if bad == "dt":
        kw["dt"] = 0.0
    elif bad == "radius":
        r = s.sph_rad.copy()
        r[3] = -1.0
        kw["sph_rad"] = r
    elif bad == "mode":
        kw["mode"] = 4
    elif bad == "adaptive_latency":
        kw["mode"], kw["lam"] = 3, 0
    elif bad == "dyn_path":
        kw["dyn_path"] = 5
    elif bad == "bin_sort":
        kw["bin_sort"] = 7
    else:
        kw["lam"] = 20
    st, ctx, msg = _create(s, **kw)
    assert st == dem.DEM_ERR_ARG
    assert msg
    if ctx:
        dem.lib().dem_destroy(ctx)


def test_calls_before_bind_report_state_error():
    _ensure_built()
    s = W.small_spheres(0, n=20)
    st, ctx, msg = _create(s)
    assert st == dem.DEM_OK
    stats = dem.StepStats()
    assert dem.lib().dem_step(ctx, 1, None, None, C.byref(stats)) == dem.DEM_ERR_STATE
    assert b"before dem_bind" in dem.lib().dem_last_error(ctx)
    F = dem.Families(None, None, None, None, None)
    assert dem.lib().dem_set_families(ctx, C.byref(F), None) == dem.DEM_ERR_STATE
    assert b"before dem_bind" in dem.lib().dem_last_error(ctx)
    dem.lib().dem_destroy(ctx)


def _set_meshes(ctx, sysm, **over):
    d = dict(n_mesh=sysm.n_mesh, n_tri=sysm.n_tri, tri_mesh=sysm.tri_mesh, tri_local=sysm.tri_local,
             origin=sysm.mesh_origin, vel=sysm.mesh_vel, omega=sysm.mesh_omega, mat=sysm.mesh_mat)
    d.update(over)
    keep = [np.ascontiguousarray(d[k], dtype=np.int32 if k in ("tri_mesh", "mat") else np.float64)
            for k in ("tri_mesh", "tri_local", "origin", "vel", "omega", "mat")]
    M = dem.Meshes(int(d["n_mesh"]), int(d["n_tri"]), *[C.c_void_p(a.ctypes.data) for a in keep])
    st = dem.lib().dem_set_meshes(ctx, C.byref(M))
    return st, dem.lib().dem_last_error(ctx).decode()


def test_meshes_grow_the_workspace_and_are_validated():
    _ensure_built()
    s = W.small_mixer(0, n=60)
    st, ctx, msg = _create(s)
    assert st == dem.DEM_OK, msg
    nb0 = C.c_int64()
    assert dem.lib().dem_workspace_size(ctx, 1000, C.byref(nb0)) == dem.DEM_OK
    st, msg = _set_meshes(ctx, s)
    assert st == dem.DEM_OK, msg
    nb1 = C.c_int64()
    assert dem.lib().dem_workspace_size(ctx, 1000, C.byref(nb1)) == dem.DEM_OK
    # per-facet buffers (two detection workspaces), facet table, pose ring
    assert nb1.value >= nb0.value + s.n_tri * (2 * 144 + 80)
    bad_mesh = s.tri_mesh.copy()
    bad_mesh[5] = 1
    nan_tri = s.tri_local.copy()
    nan_tri[3, 4] = np.nan
    for over, what in [(dict(n_mesh=5), "n_mesh"), (dict(tri_mesh=bad_mesh), "unknown mesh"),
                       (dict(mat=np.array([7])), "material"), (dict(tri_local=nan_tri), "finite"),
                       (dict(omega=np.array([[0.0, np.inf, 0.0]])), "finite")]:
        st, msg = _set_meshes(ctx, s, **over)
        assert st == dem.DEM_ERR_ARG and what in msg, (over.keys(), msg)
    # removing the meshes restores the workspace size
    assert dem.lib().dem_set_meshes(ctx, None) == dem.DEM_OK
    nb2 = C.c_int64()
    assert dem.lib().dem_workspace_size(ctx, 1000, C.byref(nb2)) == dem.DEM_OK
    assert nb2.value == nb0.value
    dem.lib().dem_destroy(ctx)
