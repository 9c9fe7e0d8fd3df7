"""Parity at the benchmark configurations' full sizes, in the launch
configuration the bench times (two streams, delayed detection), on sampled
outputs the FP64 oracle computes one by one:

* sampled rows of the active set (brute force over all spheres per row),
  bit-exact;
* forces of every contact of the sampled spheres within 1e-5;
* one integration step of the sampled owners against the oracle given all of
  their contacts.
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


def _full(name):
    if name == "config1":
        return W.config1(seed=0), 200
    if name == "config2":
        return W.config2(seed=0), 400
    if name == "config3":
        return W.config3(seed=7), 200
    if name == "config4":
        return W.config4(seed=0), 100
    if name == "mixer":
        return W.mixer(seed=0), 400
    raise ValueError(name)


def _sample_spheres(keys, Ns, rng, n):
    i = np.unique((keys >> np.uint64(32)).astype(np.int64))
    return np.sort(rng.choice(i, size=min(n, i.size), replace=False))


@pytest.mark.parametrize("name", ["config1", "config2", "config3", "config4", "mixer"])
def test_full_size_sampled_parity(dem, name):
    import torch
    s, presteps = _full(name)
    print(f"{name}: {s.n_spheres} spheres, {s.n_owners} owners", flush=True)
    ctx = dem.DemContext(s, mode="fixed", k=10, lam=5, capacity=(4 if name == "config4" else 8) * s.n_spheres)
    ctx.set_state()
    dyn, kin = torch.cuda.Stream(), torch.cuda.Stream()
    ctx.step(presteps, dyn=dyn, kin=kin)
    ctx.detect_contacts(s.margin)
    keys, hist = ctx.get_contacts()
    g = ctx.get_state()
    st = {"X": g["X"], "q": g["q"], "V": g["V"].astype(np.float64), "W": g["W"].astype(np.float64)}
    o = oracle.Oracle(s)
    rng = np.random.default_rng(1)
    nrow = 24 if name == "config4" else 60
    sample = _sample_spheres(keys, s.n_spheres, rng, nrow)
    # also a few spheres with no contact
    sample = np.unique(np.r_[sample, rng.choice(s.n_spheres, 8, replace=False)])
    if s.n_tri > 0:
        # and spheres touching the impeller's facets
        kj0 = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
        fi = np.unique((keys >> np.uint64(32)).astype(np.int64)[kj0 >= s.n_spheres + s.n_walls])
        print(f"{name}: {fi.size} spheres with facet contacts", flush=True)
        assert fi.size > 0
        sample = np.unique(np.r_[sample, rng.choice(fi, size=min(24, fi.size), replace=False)])
    rows = o.detect_rows(st, s.margin, sample, step=g["step"])
    ki = (keys >> np.uint64(32)).astype(np.int64)
    for i, row in zip(sample, rows):
        np.testing.assert_array_equal(keys[ki == i], row)
    # forces of every contact of the sampled owners (A side and B side)
    owners = np.unique(s.sph_owner[sample])
    kj = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    own_of = s.sph_owner
    mine = np.isin(own_of[ki], owners) | ((kj < s.n_spheres) & np.isin(own_of[np.minimum(kj, s.n_spheres - 1)], owners))
    sel = np.nonzero(mine)[0]
    ctx.forces()
    Fo, To, Fc = ctx.get_forces(keys.size)
    ref = o.forces(st, keys[sel], hist[sel].astype(np.float64), step=g["step"])
    Fn = np.linalg.norm(ref["Fc"], axis=1)
    touch = ref["touch"] > 0
    if touch.any():
        floor = 1e-3 * np.median(Fn[touch])
        rel = np.linalg.norm(Fc[sel] - ref["Fc"], axis=1) / np.maximum(Fn, floor)
        print(f"{name}: sampled {sample.size} spheres, {sel.size} contacts ({touch.sum()} touching), "
              f"max rel F err {rel.max():.2e}", flush=True)
        assert rel.max() <= 1e-5
    L1 = np.zeros(s.n_owners)
    np.add.at(L1, own_of[ki[sel]], Fn)
    sph = kj[sel] < s.n_spheres
    np.add.at(L1, own_of[kj[sel][sph]], Fn[sph])
    ferr = np.linalg.norm(Fo[owners] - ref["Fo"][owners], axis=1)
    assert np.all(ferr <= 1e-5 * np.maximum(L1[owners], 1e-12) + 1e-12 * s.own_mass[owners])


def test_config1_bench_configuration_deterministic_and_exact(dem):
    """The bench's headline run (1 M spheres, k = 10 on a second stream) is
    deterministic and equals every-step detection bit for bit."""
    import torch
    s = W.config1(seed=0)
    outs = []
    for mode in ("fixed", "every"):
        c = dem.DemContext(s, mode=mode, k=10, lam=5, capacity=8 * s.n_spheres)
        c.set_state()
        c.step(300, dyn=torch.cuda.Stream(), kin=torch.cuda.Stream())
        outs.append(c.get_state())
        c.close()
    for k in ("X", "V", "W"):
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
