"""Learned neighbor proposal (oracle; test infrastructure only).

The paper ranks neighbors by correlation and notes that no exact embedding of
the correlation metric exists for the Gneiting class (Sec. "Correlation-based
Vecchia neighbor selection"), so its cover tree searches the metric directly.
This module is the FP64 reference for a learned shortcut to that search:

  * features: standardised coordinates and time plus the five log
    hyperparameters that shape the correlation (log a, log c, log alpha,
    log beta, log gamma), each minus a fixed centre;
  * an MLP 8 -> 64 -> 64 -> 64 -> 16 with ReLU hidden layers (parameters
    packed as W1[8,64], b1[64], W2[64,64], b2[64], W3[64,64], b3[64],
    W4[64,16], b4[16], row-major, h_out = h_in W + b);
  * a pairwise logistic contrastive loss: rows come in groups of
    1 + npos + nneg (query, exact neighbors, non-neighbors); with
    d = |e_q - e_j|^2 the group's loss is the mean over (p, n) of
    softplus((d_p - d_n) / tau);
  * Adam;
  * the proposal search: for query i, the window is every earlier point of the
    last L+1 time slabs whose grid cell (side h) is within r cells of the
    query's in x and in y, r the smallest radius in 1..rmax at which those
    cells hold at least wmin points of the L+1 slabs (all of them, later points
    of the query's own slab included), else rmax. The ncand window points of
    smallest embedding distance (FP32, fixed order, ties to the lower index)
    -- or, without a network, of smallest spatial distance (FP64) -- are
    reranked by the exact key of the correlation search and the best m kept.
    A row whose window holds fewer than min(i, m) points or more than cmax
    points takes the exact search.

Nothing here is from the paper's text beyond the neighbor definition it
reranks to; the network, loss and window are this library's design.
"""
from __future__ import annotations

import numpy as np

from . import neighbors as NB

IN, HID, OUT = 8, 64, 16
SHAPES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("W4", (HID, OUT)), ("b4", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params):
    out = {}
    o = 0
    for name, shp in SHAPES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(params[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(params, X):
    """Embeddings E [R, 16] and the post-activation hidden layers."""
    p = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"] + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"] + p["b2"], 0.0)
    h3 = np.maximum(h2 @ p["W3"] + p["b3"], 0.0)
    E = h3 @ p["W4"] + p["b4"]
    return E, (X, h1, h2, h3)


def backward(params, cache, dE):
    """Gradient of sum(dE * E) with respect to the packed parameters."""
    p = unpack(params)
    X, h1, h2, h3 = cache
    dE = np.asarray(dE, dtype=np.float64)
    g = {"W4": h3.T @ dE, "b4": dE.sum(0)}
    d3 = (dE @ p["W4"].T) * (h3 > 0)
    g["W3"] = h2.T @ d3
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"].T) * (h2 > 0)
    g["W2"] = h1.T @ d2
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"].T) * (h1 > 0)
    g["W1"] = X.T @ d1
    g["b1"] = d1.sum(0)
    return pack(g)


def _softplus(x):
    return np.logaddexp(0.0, x)


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def pair_loss(E, npos, nneg, tau):
    """Per-group losses [B] and dE [R, 16] (gradient of the sum of group losses)."""
    E = np.asarray(E, dtype=np.float64)
    G = 1 + npos + nneg
    B = E.shape[0] // G
    Eg = E[:B * G].reshape(B, G, OUT)
    q = Eg[:, :1, :]
    diff = q - Eg[:, 1:, :]                      # [B, G-1, 16]
    d = (diff * diff).sum(-1)                    # [B, G-1]
    dp, dn = d[:, :npos], d[:, npos:]
    z = (dp[:, :, None] - dn[:, None, :]) / tau  # [B, npos, nneg]
    scale = 1.0 / (npos * nneg)
    loss = _softplus(z).sum((1, 2)) * scale
    s = _sigmoid(z) * (scale / tau)
    gdp = s.sum(2)                               # dL/dd_p
    gdn = -s.sum(1)                              # dL/dd_n
    gd = np.concatenate([gdp, gdn], axis=1)      # [B, G-1]
    # d = |q - e_j|^2: dd/dq = 2 diff, dd/de_j = -2 diff
    dE = np.zeros_like(Eg)
    dE[:, 0, :] = (2.0 * gd[:, :, None] * diff).sum(1)
    dE[:, 1:, :] = -2.0 * gd[:, :, None] * diff
    out = np.zeros_like(E)
    out[:B * G] = dE.reshape(B * G, OUT)
    return loss, out


def adam(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


HYPER = ("a", "c", "alpha", "beta", "gamma")


def features(sx, sy, t, kern, centre):
    """Inputs [n, 8]: centre = (cx, cy, ct, s_space, s_time, la, lc, lalpha, lbeta, lgamma)."""
    cx, cy, ct, ss, st = centre[:5]
    X = np.empty((sx.shape[0], IN))
    X[:, 0] = (sx - cx) / ss
    X[:, 1] = (sy - cy) / ss
    X[:, 2] = (t - ct) / st
    for c, name in enumerate(HYPER):
        X[:, 3 + c] = np.log(kern[name]) - centre[5 + c]
    return X


def grid_cells(sx, sy, h):
    """Cell columns and rows: truncation of (v - min) * (1/h), clamped to the grid."""
    x0, y0 = sx.min(), sy.min()
    ih = 1.0 / h
    gx = int((sx.max() - x0) * ih) + 1
    gy = int((sy.max() - y0) * ih) + 1
    cx = np.clip(((sx - x0) * ih).astype(np.int64), 0, gx - 1)
    cy = np.clip(((sy - y0) * ih).astype(np.int64), 0, gy - 1)
    return cx, cy


def cell_count(t, cx, cy, i, L, r):
    """Points of the slabs t_i - L .. t_i (whole slabs) within r cells of the query."""
    lo = int(np.searchsorted(t, t[i] - L, side="left"))
    hi = int(np.searchsorted(t, t[i], side="right"))
    cheb = np.maximum(np.abs(cx[lo:hi] - cx[i]), np.abs(cy[lo:hi] - cy[i]))
    return int((cheb <= r).sum())


def radius(t, cx, cy, i, L, wmin, rmax):
    """Smallest r in 1..rmax whose cells hold at least wmin points of the slabs
    t_i - L .. t_i (counting whole slabs), else rmax."""
    for r in range(1, rmax + 1):
        if cell_count(t, cx, cy, i, L, r) >= wmin:
            return r
    return rmax


def window(t, cx, cy, i, L, r=1):
    """Earlier points of the last L+1 slabs within r cells of the query (sorted)."""
    t0 = t[i] - L
    lo = int(np.searchsorted(t, t0, side="left"))
    js = np.arange(lo, i)
    ok = (np.abs(cx[js] - cx[i]) <= r) & (np.abs(cy[js] - cy[i]) <= r)
    return js[ok]


def emb_dist32(E, i, js):
    """|e_i - e_j|^2 in FP32, summed in dimension order, each product rounded."""
    e = np.asarray(E, dtype=np.float32)
    acc = np.zeros(js.shape[0], dtype=np.float32)
    for k in range(OUT):
        d = (e[i, k] - e[js, k]).astype(np.float32)
        acc = (acc + (d * d).astype(np.float32)).astype(np.float32)
    return acc


def propose(kern, sx, sy, t, m, E, ncand, h, L, cmax, rows=None, wmin=0, rmax=1):
    """Proposal neighbor rows [len(rows), m] (-1 padded) and the fallback mask."""
    n = sx.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    cx, cy = grid_cells(sx, sy, h)
    max_lag = int(t[-1] - t[0]) if n else 0
    tabs = NB.lag_tables(kern, max_lag)
    out = np.full((rows.shape[0], m), -1, dtype=np.int32)
    fb = np.zeros(rows.shape[0], dtype=bool)
    for r, i in enumerate(rows):
        rad = radius(t, cx, cy, i, L, wmin, rmax)
        js = window(t, cx, cy, i, L, rad)
        if js.shape[0] < min(i, m) or js.shape[0] > cmax:
            fb[r] = True
            ex = NB.brute_force(kern, sx, sy, t, m, rows=[i])[0]
            out[r] = ex
            continue
        if js.shape[0] == 0:
            continue
        if E is None:
            dx = sx[js] - sx[i]
            dy = sy[js] - sy[i]
            score = dx * dx + dy * dy
        else:
            score = emb_dist32(E, i, js)
        cand = js[np.lexsort((js, score))[:ncand]]
        k = NB.keys(kern, tabs, sx, sy, t, i, cand)
        order = np.lexsort((cand, -k))[:m]
        out[r, :order.shape[0]] = cand[order]
    return out, fb


def recall(prop, exact):
    """Share of the exact neighbor entries (excluding -1 padding) found in the proposal."""
    hit = tot = 0
    for a, b in zip(prop, exact):
        sb = set(int(x) for x in b if x >= 0)
        tot += len(sb)
        hit += len(sb & set(int(x) for x in a if x >= 0))
    return hit / max(tot, 1)
