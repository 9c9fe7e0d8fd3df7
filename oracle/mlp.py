"""FP64 oracle of the learned contact-detection interval (test infrastructure).

The paper adapts the update bound n_max from timing history (Sec. 2.1); the
learned part replaces that with a small network that predicts, per feature
cell, how many more steps a freshly detected active set stays complete.
This module is the plain definition of what the GPU kernels compute:

* ``features``: the six per-cell features of a state relative to the state
  at the previous detection (definitions below; cells of edge 8 (r_max + m));
* ``labels``: the first step at which a true contact touching a cell is
  missing from a set detected with the margin;
* ``forward`` / ``loss_and_grad`` / ``adam_step``: the 6-32-32-1 tanh MLP,
  the expectile loss and the Adam update, in float64 with numpy.

Parameter layout (row-major, out x in): W1[32x6], b1[32], W2[32x32], b2[32],
W3[1x32], b3[1] -- 1313 values.
"""
from __future__ import annotations

import math

import numpy as np

H = 32
NF = 6
NPARAM = H * NF + H + H * H + H + H + 1
K_CAP = 1024.0


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H].reshape(1, H); o += H
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def forward(p, X):
    """y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 for every row x of X."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = (h2 @ W3.T)[:, 0] + b3[0]
    return y, (X, h1, h2)


def expectile_loss(y, T, tau):
    """Mean asymmetric squared error: weight 1 - tau where the prediction is
    above the target, tau where it is at or below (tau < 0.5 favours
    under-prediction)."""
    r = y - np.asarray(T, dtype=np.float64)
    w = np.where(r > 0.0, 1.0 - tau, tau)
    return float(np.mean(w * r * r))


def loss_and_grad(p, X, T, tau):
    """Loss and its gradient with respect to the 1313 parameters
    (back-propagation through the two tanh layers)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (X, h1, h2) = forward(p, X)
    n = X.shape[0]
    r = y - np.asarray(T, dtype=np.float64)
    w = np.where(r > 0.0, 1.0 - tau, tau)
    loss = float(np.mean(w * r * r))
    g = 2.0 * w * r / n                       # dL/dy
    dW3 = (g @ h2)[None, :]
    db3 = np.array([g.sum()])
    d2 = (g[:, None] * W3) * (1.0 - h2 * h2)  # dL/d(pre-activation 2)
    dW2 = d2.T @ h1
    db2 = d2.sum(0)
    d1 = (d2 @ W2) * (1.0 - h1 * h1)
    dW1 = d1.T @ X
    db1 = d1.sum(0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


def grad_term_magnitudes(p, X, T, tau):
    """Per parameter, the summed magnitudes of the per-sample terms its
    gradient adds up (back-propagation with every factor replaced by its
    magnitude, and every inner sum by the sum of its terms' magnitudes):
    the scale against which a float32 evaluation's rounding is bounded."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (X, h1, h2) = forward(p, X)
    n = X.shape[0]
    r = y - np.asarray(T, dtype=np.float64)
    w = np.where(r > 0.0, 1.0 - tau, tau)
    g = np.abs(2.0 * w * r / n)
    aX, a1, a2 = np.abs(X), np.abs(h1), np.abs(h2)
    dW3 = (g @ a2)[None, :]
    db3 = np.array([g.sum()])
    d2 = (g[:, None] * np.abs(W3)) * (1.0 - h2 * h2)
    dW2 = d2.T @ a1
    db2 = d2.sum(0)
    d1 = (d2 @ np.abs(W2)) * (1.0 - h1 * h1)
    dW1 = d1.T @ aX
    db1 = d1.sum(0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), returning new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# features and labels
# ---------------------------------------------------------------------------

def feature_grid(sysm):
    """Feature cells: cubes of edge E = 8 (r_max + m) -- four times the
    smallest edge a detection bin may have, 2 (r_max + m) -- tiling the
    domain box from its low corner, ceil(extent / E) cells per axis (at
    least one).  Returns (low corner, E, cells per axis)."""
    E = 8.0 * (float(np.max(sysm.sph_rad)) + sysm.margin)
    if not E > 0.0:
        E = 1.0
    lo = np.asarray(sysm.domain_lo, dtype=np.float64)
    hi = np.asarray(sysm.domain_hi, dtype=np.float64)
    n = np.maximum(np.ceil((hi - lo) / E).astype(np.int64), 1)
    return lo, E, n


def owner_cells(sysm, X):
    """Cell id of each owner centre, (cz ny + cy) nx + cx, a centre outside
    the box taken to the nearest cell."""
    lo, edge, nf = feature_grid(sysm)
    c = np.floor((np.asarray(X) - lo) * (1.0 / edge))
    c = np.clip(c, 0, nf - 1).astype(np.int64)
    return (c[:, 2] * nf[1] + c[:, 1]) * nf[0] + c[:, 0]


def features(sysm, X, V, Xs, Vs, tau_steps):
    """Per occupied cell (ascending cell id), from the owners whose centre
    lies in it, with K = 1024 (the label horizon), m the margin, h the step, tau the steps since
    the snapshot (Xs, Vs):
      f1 log1p(|max V - min V| h K / m)   (componentwise range of velocities)
      f2 log1p(max|V - Vs| K^2 h / (2 max(tau,1) m))
      f3 sum of the owners' sphere volumes / cell volume
      f4 tau / K
      f5 log1p(max|V| h K / m)
      f6 log1p(max|X - Xs| / m)
    Returns (cell ids, features[n,6])."""
    h, m = sysm.dt, (sysm.margin if sysm.margin > 0 else 1e-6)
    cells = owner_cells(sysm, X)
    lo, edge, nf = feature_grid(sysm)
    vol_owner = np.zeros(sysm.n_owners)
    np.add.at(vol_owner, sysm.sph_owner, 4.0 / 3.0 * math.pi * sysm.sph_rad ** 3)
    ids = np.unique(cells)
    out = np.zeros((ids.size, NF))
    t = max(float(tau_steps), 1.0)
    for k, c in enumerate(ids):
        sel = cells == c
        v = V[sel]
        spread = np.linalg.norm(v.max(0) - v.min(0))
        dv = np.linalg.norm(V[sel] - Vs[sel], axis=1).max()
        va = np.linalg.norm(v, axis=1).max()
        dx = np.linalg.norm(X[sel] - Xs[sel], axis=1).max()
        out[k] = [math.log1p(spread * h * K_CAP / m),
                  math.log1p(dv * K_CAP * K_CAP * h / (2.0 * t * m)),
                  vol_owner[sel].sum() / edge ** 3,
                  tau_steps / K_CAP,
                  math.log1p(va * h * K_CAP / m),
                  math.log1p(dx / m)]
    return ids, out


def first_miss_per_cell(sysm, label_keys, true_keys, owner_cell, t, first):
    """Lowers first[cell] to t for every true contact absent from the label
    set, on the cells of both owners (sphere-wall contacts: the sphere's)."""
    missing = np.setdiff1d(true_keys, label_keys, assume_unique=True)
    i = (missing >> np.uint64(32)).astype(np.int64)
    j = (missing & np.uint64(0xFFFFFFFF)).astype(np.int64)
    for a in owner_cell[sysm.sph_owner[i]]:
        first[a] = min(first[a], t)
    for b in owner_cell[sysm.sph_owner[j[j < sysm.n_spheres]]]:
        first[b] = min(first[b], t)
    return first
