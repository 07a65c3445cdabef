"""Covariance localisation (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4 names two localisations: the local analysis the paper develops, and
covariance localisation (CL), in which the prediction covariance is tapered
by a Schur product with a distance-based correlation matrix, which raises its
rank and removes spurious long-range correlations; it does not write CL out.
Reading used here, kept inside the same domains and observation regions so
that the domains stay independent:

* per domain, over its node patch (owned nodes and the corners of its
  observation subapertures), the tapered prior covariance
  P_loc = rho_xx o (kappa X'_P X'_P^T), kappa = rho / (m - 1) (the inflated
  ensemble covariance), rho_xx the Gaspari-Cohn function of the node-node
  distance over c (c the taper half width in pitches; c = 0: no taper);
* the slope operator applied to it exactly: with the slopes whitened by the
  noise (Dt = R_l^{-1/2} D_l, dt = R_l^{-1/2} d, R = s diag(r)),
  S = Dt P_loc Dt^T + I and the gain of the owned rows
  K = P_loc[own, :] Dt^T S^{-1};
* mean x_a = x_b + K dt; anomalies by the deterministic EnKF (Sakov & Oke
  2008), X'_a = sqrt(rho) (X'_own - K Yt / 2), Yt = Dt X'_P: the transform of
  the local analysis has no counterpart for a tapered covariance;
* the owned rows are gathered by concatenation; the Sec. 4.4 piston step may
  follow.

Tapering the slope-space covariances instead (rho_yy o (Yt Yt^T),
rho_xy o (X' Yt^T)) cuts the phase from the slopes that integrate to it and
diverges on these workloads.  With the taper off the mean is the local
analysis's (Sherman-Morrison-Woodbury); the anomalies then differ from the
transform's at second order in the gain.  The observation weights of the
local analysis (the taper on Sigma_w^{-1/2}) are not applied: c tapers the
covariance instead.
"""
from __future__ import annotations

import numpy as np

from . import blend as BL
from . import geometry as geo
from . import letkf as ol


def node_correlation(geom, nodes, c) -> np.ndarray:
    """rho_xx over the given nodes."""
    pos = geom.node_coords()[nodes].astype(np.float64)
    if c <= 0.0:
        return np.ones((len(nodes), len(nodes)))
    dist = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
    return geo.gaspari_cohn(dist / c)


def local_operators(geom, dom, r_diag, params):
    """(patch nodes, whitened local slope operator Dt (p_l x patch))."""
    P = BL.patch_nodes(geom, dom)
    D = np.zeros((len(dom.obs), geom.n_nodes))
    idx = geom.node_index
    ps = geom.n_subaps
    for row, s in enumerate(dom.obs):
        k = s % ps
        i, j = geom.subaps[k]
        a, b, c, d = idx[i, j], idx[i, j + 1], idx[i + 1, j], idx[i + 1, j + 1]
        if s < ps:   # x-slope
            D[row, [a, b, c, d]] += [-0.5, 0.5, -0.5, 0.5]
        else:        # y-slope
            D[row, [a, b, c, d]] += [-0.5, -0.5, 0.5, 0.5]
    w = 1.0 / np.sqrt(params.r_scale * np.asarray(r_diag, np.float64)[dom.obs])
    return P, w[:, None] * D[:, P]


def local_update(geom, dom, xb, Xp, d, r_diag, params: ol.Params):
    """Analysis members of the owned rows of one domain."""
    P, Dt = local_operators(geom, dom, r_diag, params)
    m = Xp.shape[1]
    kap = params.rho / (m - 1)
    XP = Xp[P]
    Ploc = node_correlation(geom, P, params.taper_c) * (kap * XP @ XP.T)
    S = Dt @ Ploc @ Dt.T + np.eye(len(dom.obs))
    own = np.searchsorted(P, dom.owned)
    K = np.linalg.solve(S, Dt @ Ploc[:, own]).T
    dt = d[dom.obs] / np.sqrt(params.r_scale * np.asarray(r_diag, np.float64)[dom.obs])
    xa = xb[dom.owned] + K @ dt
    return xa[:, None] + np.sqrt(params.rho) * (XP[own] - 0.5 * K @ (Dt @ XP))


def analysis(geom, doms, Xb, y, r_diag, params: ol.Params) -> np.ndarray:
    Xb = np.asarray(Xb, np.float64)
    xb, Xp = ol.ensemble_stats(Xb)
    d = np.asarray(y, np.float64) - geo.apply_slopes(geom, xb)
    Xa = np.empty_like(Xb)
    for dom in doms:
        Xa[dom.owned] = local_update(geom, dom, xb, Xp, d, r_diag, params)
    return Xa


def step(geom, doms, Xa_prev, V, y, r_diag, params: ol.Params) -> np.ndarray:
    """One frame with the CL analysis; the piston step when params.piston."""
    Xa = analysis(geom, doms, ol.forecast(Xa_prev, V, params.a), y, r_diag, params)
    if params.piston:
        from . import piston
        Xa = piston.remove(geom, doms, Xa, y)
    return Xa
