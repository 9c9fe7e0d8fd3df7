"""The FP32 prefilter of the detection walk never rejects a pair that the
exact FP64 predicate accepts.

The walk first compares an FP32 distance, computed from candidate copies
rounded to float32 relative to the grid origin, with the pair threshold
plus a rounding slack 8 u (M_i + M_j) + 16 u T + 1e-12 m (u = 2^-24, M the
largest coordinate magnitude of a sphere, T the threshold).  This test
replays that float32 arithmetic operation by operation (numpy rounds every
float32 operation; nothing is fused) on pairs placed just inside the exact
threshold, with coordinates up to 100 m from the origin, radii from 0.1 to
10 mm and margins up to 1 mm, and checks that none of them is rejected.
"""
import numpy as np

F = np.float32


def _prefilter_rejects(ci, cj, ri, rj, m):
    """float32 replay of the walk's prefilter; ci, cj: float32 copies [n,3]."""
    twom = F(2.0 * m) if np.isscalar(m) else (2.0 * m).astype(F)
    Mi = np.maximum(np.abs(ci[:, 0]), np.maximum(np.abs(ci[:, 1]), np.abs(ci[:, 2])))
    Mj = np.maximum(np.abs(cj[:, 0]), np.maximum(np.abs(cj[:, 1]), np.abs(cj[:, 2])))
    dx, dy, dz = ci[:, 0] - cj[:, 0], ci[:, 1] - cj[:, 1], ci[:, 2] - cj[:, 2]
    T32 = (ri + rj) + twom
    tf = T32 + ((F(4.77e-7) * (Mi + Mj) + F(9.54e-7) * T32) + F(1e-12))
    d2 = (dx * dx + dy * dy) + dz * dz
    assert d2.dtype == F and tf.dtype == F
    return d2 > tf * tf


def _exact_hit(xi, xj, ri, rj, m):
    d = xi - xj
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    T = (ri.astype(np.float64) + rj.astype(np.float64)) + 2.0 * m
    return d2 < T * T


def test_prefilter_never_rejects_an_exact_pair():
    rng = np.random.default_rng(0)
    n = 400_000
    for scale in (0.05, 1.0, 100.0):
        lo = rng.uniform(-5, 5, size=3)
        xi = lo + rng.uniform(0, scale, size=(n, 3))
        ri = rng.uniform(1e-4, 1e-2, size=n).astype(F)
        rj = rng.uniform(1e-4, 1e-2, size=n).astype(F)
        m = rng.uniform(0, 1e-3, size=n)
        m[: n // 4] = 0.0
        T = (ri.astype(np.float64) + rj.astype(np.float64)) + 2.0 * m
        u = rng.normal(size=(n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        # distances just inside the threshold, down to relative 1e-15
        shrink = 10.0 ** rng.uniform(-15, -3, size=n)
        xj = xi - (T * (1.0 - shrink))[:, None] * u
        hit = _exact_hit(xi, xj, ri, rj, m)
        assert hit.mean() > 0.9
        ci = (xi - lo).astype(F)
        cj = (xj - lo).astype(F)
        rej = _prefilter_rejects(ci, cj, ri, rj, m)
        assert not np.any(hit & rej), int(np.sum(hit & rej))


def test_prefilter_rejects_most_of_what_is_clearly_outside():
    """The slack is small: pairs 1 % beyond the threshold are rejected."""
    rng = np.random.default_rng(1)
    n = 100_000
    lo = np.zeros(3)
    xi = rng.uniform(0, 1.0, size=(n, 3))
    ri = rng.uniform(2e-3, 3e-3, size=n).astype(F)
    rj = rng.uniform(2e-3, 3e-3, size=n).astype(F)
    m = 2e-4
    T = (ri.astype(np.float64) + rj.astype(np.float64)) + 2.0 * m
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    xj = xi - (T * 1.01)[:, None] * u
    rej = _prefilter_rejects((xi - lo).astype(F), (xj - lo).astype(F), ri, rj, m)
    assert rej.all()
