"""Differential-piston removal after the gather (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each local analysis is blind to the piston of its own domain (the slopes do
not see a constant phase), so the concatenated estimate carries a different
unknown piston per domain; the paper removes these inside the loop with a
least-squares fit that minimises the discontinuities between neighbouring
domains over the whole pupil (Sec. 4.4).  Reading used here: the pistons pi
(one per domain) minimise the slope misfit of the piston-corrected analysis
mean on the subapertures whose four corners are not all in one domain (the
only slopes a differential piston changes):

    pi = argmin || D_B (x_a + P pi) - y_B ||^2,   P[node, domain] = 1 if owned,

with the minimum-norm solution (pistons sum to zero on every connected set of
domains: a common piston is not measurable).  Every member of a domain is
shifted by its piston, so the analysis mean moves and the anomalies do not.
The fit is unweighted, as in the paper (noise propagation is left out there).

The adjoint of the step (for the gradient of a loss through it), with
pi = M^+ P^T D^T (y - D x_a) and M = P^T D^T D P:
    X_a_bar <- Z_bar - (1/m) (D^T D P M^+ P^T Z_bar 1) 1^T
for the adjoint Z_bar of the corrected ensemble.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo


def border_system(geom, doms):
    """(A, rows): A is the dense (r, n_domains) matrix D_B P of the slopes of
    the border subapertures (x then y slope of each, ascending subaperture),
    rows their global slope indices."""
    own = geo.owner_map(geom, doms)
    idx = geom.node_index
    ps = geom.n_subaps
    nd = len(doms)
    A, rows = [], []
    for k, (i, j) in enumerate(geom.subaps):
        a, b, c, d = idx[i, j], idx[i, j + 1], idx[i + 1, j], idx[i + 1, j + 1]
        if len({own[a], own[b], own[c], own[d]}) == 1:
            continue
        for comp, coef in ((0, ((a, -0.5), (b, 0.5), (c, -0.5), (d, 0.5))),
                           (1, ((a, -0.5), (b, -0.5), (c, 0.5), (d, 0.5)))):
            row = np.zeros(nd)
            for node, cf in coef:
                row[own[node]] += cf
            A.append(row)
            rows.append(comp * ps + k)
    return np.array(A).reshape(-1, nd), np.array(rows, dtype=np.int64)


def pistons(geom, doms, x_mean, y) -> np.ndarray:
    """The least-squares per-domain pistons of the analysis mean x_mean."""
    A, rows = border_system(geom, doms)
    if A.shape[0] == 0:
        return np.zeros(len(doms))
    resid = np.asarray(y, np.float64)[rows] - geo.apply_slopes(geom, np.asarray(x_mean, np.float64))[rows]
    return np.linalg.lstsq(A, resid, rcond=None)[0]


def remove(geom, doms, Xa, y) -> np.ndarray:
    """The analysis ensemble with every member of domain d shifted by pi_d."""
    Xa = np.asarray(Xa, np.float64)
    pi = pistons(geom, doms, Xa.mean(axis=1), y)
    own = geo.owner_map(geom, doms)
    return Xa + pi[own][:, None]


def remove_adjoint(geom, doms, Z_bar) -> np.ndarray:
    """Adjoint of `remove` with respect to its input ensemble."""
    Z_bar = np.asarray(Z_bar, np.float64)
    A, _ = border_system(geom, doms)
    own = geo.owner_map(geom, doms)
    m = Z_bar.shape[1]
    if A.shape[0] == 0:
        return Z_bar.copy()
    s = np.zeros(len(doms))
    np.add.at(s, own, Z_bar.sum(axis=1))
    t = np.linalg.pinv(A.T @ A) @ s
    xbar = -geo.apply_slopes_adjoint(geom, geo.apply_slopes(geom, t[own]))
    return Z_bar + xbar[:, None] / m


__all__ = ["border_system", "pistons", "remove", "remove_adjoint"]
