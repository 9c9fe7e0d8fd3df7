"""Pins of the FP64 MLP / feature / label oracle (CPU only)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import mlp


def _rand(seed, n=257):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, size=mlp.NPARAM)
    X = rng.normal(0, 1.0, size=(n, mlp.NF))
    T = rng.normal(0, 1.0, size=n)
    return p, X, T


def _torch_net(p):
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    ts = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (W1, b1, W2, b2, W3, b3)]
    return ts


def _torch_forward(ts, X):
    W1, b1, W2, b2, W3, b3 = ts
    x = torch.tensor(X, dtype=torch.float64)
    h1 = torch.tanh(torch.nn.functional.linear(x, W1, b1))
    h2 = torch.tanh(torch.nn.functional.linear(h1, W2, b2))
    return torch.nn.functional.linear(h2, W3, b3)[:, 0]


def test_parameter_count():
    assert mlp.NPARAM == 1313


def test_forward_matches_torch_linear_tanh():
    p, X, _ = _rand(0)
    y, _ = mlp.forward(p, X)
    yt = _torch_forward(_torch_net(p), X).detach().numpy()
    np.testing.assert_allclose(y, yt, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("tau", [0.05, 0.5, 0.9])
def test_gradient_matches_torch_autograd(tau):
    p, X, T = _rand(1)
    loss, g = mlp.loss_and_grad(p, X, T, tau)
    ts = _torch_net(p)
    y = _torch_forward(ts, X)
    r = y - torch.tensor(T)
    w = torch.where(r > 0, torch.tensor(1.0 - tau, dtype=torch.float64), torch.tensor(tau, dtype=torch.float64))
    lt = torch.mean(w * r * r)
    lt.backward()
    gt = np.concatenate([t.grad.numpy().ravel() for t in ts])
    assert abs(loss - lt.item()) <= 1e-13 * abs(loss)
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_gradient_matches_finite_differences():
    p, X, T = _rand(2, n=40)
    tau = 0.05
    _, g = mlp.loss_and_grad(p, X, T, tau)
    rng = np.random.default_rng(3)
    idx = rng.choice(mlp.NPARAM, size=40, replace=False)
    for k in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        yp, _ = mlp.forward(pp, X)
        ym, _ = mlp.forward(pm, X)
        fd = (mlp.expectile_loss(yp, T, tau) - mlp.expectile_loss(ym, T, tau)) / (2 * e)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9


def test_expectile_half_is_half_mse():
    p, X, T = _rand(4)
    y, _ = mlp.forward(p, X)
    assert abs(mlp.expectile_loss(y, T, 0.5) - 0.5 * np.mean((y - T) ** 2)) < 1e-15


def test_adam_matches_torch():
    p, X, T = _rand(5)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(6)
    for t in range(1, 6):
        g = rng.normal(0, 1, size=p.size)
        p, m, v = mlp.adam_step(p, g, m, v, t)
        opt.zero_grad()
        pt.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_features_closed_form():
    """Three owners in one cell with known motion since the snapshot."""
    s = W.small_spheres(0, n=3, walls=False)
    c0 = W.snap_pos(np.array([0.0012, 0.0011, 0.0013]))
    X = np.array([c0, c0 + 0.0005, c0 - 0.0004])
    Xs = X - np.array([[1e-5, 0, 0], [0, 2e-5, 0], [0, 0, 0]])
    V = np.array([[0.1, 0.0, 0.0], [0.0, -0.2, 0.0], [0.0, 0.0, 0.3]])
    Vs = np.zeros((3, 3))
    ids, f = mlp.features(s, X, V, Xs, Vs, tau_steps=8)
    assert ids.size == 1
    h, m, K = s.dt, s.margin, mlp.K_CAP
    lo, edge, nf = mlp.feature_grid(s)
    spread = math.sqrt(0.1 ** 2 + 0.2 ** 2 + 0.3 ** 2)
    vol = (4 / 3 * math.pi * s.sph_rad ** 3).sum() / edge ** 3
    exp = [math.log1p(spread * h * K / m), math.log1p(0.3 * K * K * h / (2 * 8 * m)), vol, 8 / K,
           math.log1p(0.3 * h * K / m), math.log1p(2e-5 / m)]
    np.testing.assert_allclose(f[0], exp, rtol=1e-12)


def test_labels_first_miss_at_touch_time():
    """Two spheres outside the label margin closing at speed v: the first
    missing true contact appears at the step where the gap closes."""
    import oracle
    r, gap, v = 0.005, 0.002, 1.0
    s = W.assemble(np.full(2, -1), np.array([[-r - gap / 2, 0, 0], [r + gap / 2, 0, 0]]), W._qid(2),
                   np.array([[v / 2, 0, 0], [-v / 2, 0, 0]]), np.zeros((2, 3)), [], r, None, W.concat_walls(),
                   W.materials(), (0, 0, 0), 1e-5, 0.0002, -0.1 * np.ones(3), 0.1 * np.ones(3))
    o = oracle.Oracle(s)
    st = o.state()
    lab = o.detect(st, s.margin)
    assert lab.size == 0
    cells = mlp.owner_cells(s, st["X"])
    first = np.full(int(np.prod(mlp.feature_grid(s)[2])), 10 ** 9)
    acs = None
    step = 0
    for t in range(1, 400):
        st, acs, _, step = o.run(st, 1, mode="every", acs=acs, step=step)
        true = o.detect(st, 0.0, step=step)
        mlp.first_miss_per_cell(s, lab, true, cells, t, first)
        if first.min() < 10 ** 9:
            break
    gap_exact = abs(s.X[1, 0] - s.X[0, 0]) - 2 * s.sph_rad[0]
    t_touch = math.floor(gap_exact / (v * s.dt)) + 1
    assert first.min() == t_touch


def test_grad_term_magnitudes_bound_the_gradient():
    """The summed term magnitudes bound the gradient component by component
    (|sum| <= sum of |terms|), equal it where no term changes sign (a
    single sample with positive inputs, weights and residual), and scale
    linearly with the number of identical samples."""
    rng = np.random.default_rng(3)
    p = rng.normal(0, 0.3, size=mlp.NPARAM)
    X = rng.normal(0, 1.0, size=(50, mlp.NF))
    T = rng.normal(0, 1.0, size=50)
    _, g = mlp.loss_and_grad(p, X, T, 0.05)
    A = mlp.grad_term_magnitudes(p, X, T, 0.05)
    assert np.all(np.abs(g) <= A * (1 + 1e-12) + 1e-300)
    pp = np.abs(p)
    x1 = np.abs(X[:1])
    t1 = np.array([-5.0])   # prediction above the target: positive residual
    _, g1 = mlp.loss_and_grad(pp, x1, t1, 0.05)
    A1 = mlp.grad_term_magnitudes(pp, x1, t1, 0.05)
    np.testing.assert_allclose(np.abs(g1), A1, rtol=1e-12, atol=1e-300)
    A3 = mlp.grad_term_magnitudes(p, np.repeat(X[:1], 3, 0), np.repeat(T[:1], 3), 0.05)
    Ab = mlp.grad_term_magnitudes(p, X[:1], T[:1], 0.05)
    np.testing.assert_allclose(A3, Ab, rtol=1e-12)   # (the mean over n: 3 equal samples, 1/3 each)
