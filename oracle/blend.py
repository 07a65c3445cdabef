"""Blend-mode gather (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.2 forms X_a by concatenating the owned rows of the local analyses, and
Sec. 4.1 asks that the updates of neighbouring domains agree at their common
border.  This variant replaces the concatenation, which the paper does not
vary, by a weighted blend of overlapping local analyses.  Reading used here:

* every domain l updates all nodes of its patch P_l (its owned nodes and the
  corners of its observation-region subapertures) with its own w and W:
  X_l(n) = x_b(n) + X'(n) w + sqrt(rho) X'(n) W;
* the slopes do not see a domain's piston, so the patches are first put on a
  common piston: pi minimises, over every node n and every pair of domains
  l, l' whose patches hold n, the squared difference of the analysis means
  (xbar_l(n) + pi_l) - (xbar_l'(n) + pi_l'); the minimum-norm solution (zero
  sum on each connected set of domains);
* the gathered ensemble is the weighted mean over the domains whose patch
  holds the node, X_a(n) = sum_l om_l(n) (X_l(n) + pi_l) / sum_l om_l(n),
  with the separable tent om_l(n) = t(d_i) t(d_j), t(d) = 1 - d / (h + 2),
  d_i (d_j) the distance in node pitches of the node's row (column) from the
  rows (columns) of domain l's b x b block (0 inside; the last block row and
  column run to the grid edge).

A node's owner gives it weight 1, so every denominator is at least 1, and on
a patch d <= h + 1, so every weight is positive.  The differential-piston
step of Sec. 4.4 is not applied after the blend (the alignment takes its
place).
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from . import letkf as ol


def _span(K, b, N):
    nb = -(-N // b)
    return K * b, (N if K == nb - 1 else (K + 1) * b - 1)


def patch_nodes(geom, dom) -> np.ndarray:
    """Ascending node indices of P_l: owned nodes and the corners of the
    observation-region subapertures."""
    idx = geom.node_index
    corners = [idx[i + di, j + dj] for i, j in dom.obs_subaps for di in (0, 1) for dj in (0, 1)]
    return np.unique(np.concatenate([dom.owned, np.asarray(corners, np.int64)]))


def weights(geom, dom, b, h, nodes) -> np.ndarray:
    """om_l(n) for the given nodes of domain l."""
    ij = geom.node_coords()[nodes]
    I, J = dom.block
    out = np.ones(len(nodes))
    for ax, K in ((0, I), (1, J)):
        lo, hi = _span(K, b, geom.n_sub)
        d = np.maximum(0, np.maximum(lo - ij[:, ax], ij[:, ax] - hi))
        out *= 1.0 - d / (h + 2.0)
    return out


def alignment(parts, n_domains) -> np.ndarray:
    """pi from the patches' analysis means: one least-squares equation
    pi_l - pi_l' = xbar_l'(n) - xbar_l(n) per shared node and pair of
    domains, minimum-norm solution.  parts[l] = (P_l, X_l)."""
    holders = {}
    for l, (P, X) in enumerate(parts):
        xm = X.mean(axis=1)
        for k, n in enumerate(P):
            holders.setdefault(int(n), []).append((l, xm[k]))
    rows, rhs = [], []
    for lst in holders.values():
        for u in range(len(lst)):
            for v in range(u + 1, len(lst)):
                row = np.zeros(n_domains)
                row[lst[u][0]], row[lst[v][0]] = 1.0, -1.0
                rows.append(row)
                rhs.append(lst[v][1] - lst[u][1])
    if not rows:
        return np.zeros(n_domains)
    return np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]


def gather(parts, weights_list, n_nodes) -> np.ndarray:
    """Aligned weighted blend of the patch analyses."""
    pi = alignment(parts, len(parts))
    m = parts[0][1].shape[1]
    num = np.zeros((n_nodes, m))
    den = np.zeros(n_nodes)
    for (P, X), om, p in zip(parts, weights_list, pi):
        num[P] += om[:, None] * (X + p)
        den[P] += om
    return num / den[:, None]


def analysis(geom, doms, Xb, y, r_diag, params: ol.Params, u_prev2=None) -> np.ndarray:
    """Local analyses of every patch, aligned and blended.  u_prev2 given: the
    closed loop's observation, y_bar = D x_b - D N u_{k-2} (Sec. 2.2)."""
    from . import delayed as DL
    Xb = np.asarray(Xb, np.float64)
    xb, Xp = ol.ensemble_stats(Xb)
    Yp = geo.apply_slopes(geom, Xp)
    d = np.asarray(y, np.float64) - DL.predicted_slopes(geom, xb, u_prev2)
    parts, oms = [], []
    for dom in doms:
        Y, dl, g = ol.local_inputs(geom, dom, Yp, d, r_diag, params)
        w, W, _, _ = ol.local_weights(Y, dl, g, params.rho)
        P = patch_nodes(geom, dom)
        _, Xl = ol.local_update(xb[P], Xp[P], w, W, params.rho)
        parts.append((P, Xl))
        oms.append(weights(geom, dom, params.b, params.h, P))
    return gather(parts, oms, geom.n_nodes)


def step(geom, doms, Xa_prev, V, y, r_diag, params: ol.Params) -> np.ndarray:
    """One frame with the blend-mode gather."""
    return analysis(geom, doms, ol.forecast(Xa_prev, V, params.a), y, r_diag, params)
