"""The local ETKF frame, written out plainly in FP64 (oracle side).

One frame k (forecast first, then the analysis that uses the slopes y_k of the
true phase at frame k) on a delay-free zonal phase state x (valid actuator
nodes, App. B with the state reduced to the current phase):

F1  Forecast (Sec. 3.1.2, member prediction equation; App. B.2 with
    A_tur = a Id):  X_b = a X_a + V, one column per member.
F2  Mean and anomalies (Sec. 3.1, empirical covariance equation):
    x_b = X_b 1 / m,  X_b' = X_b - x_b 1^T.  Slope-space anomalies and mean:
    Y_b' = D X_b', y_bar = D x_b, innovation d = y - y_bar.
L1  For each domain l (Sec. 4.2, independently): Y_l = the observation-region
    rows of the global Y_b' (the local observation operator applied to the
    global anomalies), d_l likewise, and the per-slope weight
    g = f^2 / (s r): the inverse noise variance scaled by the taper f
    (f multiplies Sigma_w^{-1/2}, Sec. 4.1) and by the noise scale s.
L2  A~ = (m-1)/rho I + Y_l^T diag(g) Y_l  (m x m, SPD; rho the multiplicative
    inflation of Hunt et al. 2007, cited in Sec. 4; rho = 1 gives the paper's
    Id + S_cz^T S_cz up to the factor (m-1)).
L3  A~ = Q Lambda Q^T (Sec. 3.1.1, EVD of the m x m matrix).
L4  w = A~^{-1} Y_l^T diag(g) d_l,  W = sqrt((m-1)/rho) A~^{-1/2}.
L5  x_a,l = x_b,l + X_l' w,  X_a,l = x_a,l 1^T + sqrt(rho) X_l' W.
G   Concatenate the owned rows of every domain (Sec. 4.2).

Two further forms of the same local update are kept as independent checks:
`local_update_smw` follows the paper's SMW form (Sec. 4.2 local update
equations and App. A, written for inflated anomalies sqrt(rho) X'), and
`local_mean_gain` the local Kalman gain form (Sec. 4.2, gain written with the
innovation factored to the right).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import geometry as geo


@dataclass
class Params:
    a: float = 0.99            # AR(1) coefficient
    rho: float = 1.05          # multiplicative inflation
    r_scale: float = 1.0       # s: R = s diag(r)
    b: int = 4                 # domain size in subapertures
    h: int = 1                 # halo in subapertures
    taper_c: float = 0.0       # Gaspari-Cohn half width in pitches, 0 = off
    piston: bool = False       # differential-piston removal after the gather (Sec. 4.4)


def forecast(Xa: np.ndarray, V: np.ndarray, a: float) -> np.ndarray:
    """F1: X_b = a X_a + V."""
    return a * np.asarray(Xa, dtype=np.float64) + np.asarray(V, dtype=np.float64)


def ensemble_stats(Xb: np.ndarray):
    """F2: member mean and anomalies (columns are members)."""
    xb = Xb.mean(axis=1)
    return xb, Xb - xb[:, None]


def local_weights(Y: np.ndarray, d: np.ndarray, g: np.ndarray, rho: float):
    """L2-L4: mean weights w and transform W of one domain.

    Y: (p_l, m) slope anomalies, d: (p_l,) innovation, g: (p_l,) weights.
    Returns (w, W, A~, eigenvalues)."""
    m = Y.shape[1]
    c = (m - 1) / rho
    A = c * np.eye(m) + Y.T @ (g[:, None] * Y)
    lam, Q = np.linalg.eigh(A)
    b = Y.T @ (g * d)
    w = Q @ ((Q.T @ b) / lam)
    W = np.sqrt(c) * (Q / np.sqrt(lam)) @ Q.T
    return w, W, A, lam


def local_update(xb_l: np.ndarray, Xp_l: np.ndarray, w: np.ndarray, W: np.ndarray,
                 rho: float):
    """L5: analysis mean and members of the owned rows."""
    xa = xb_l + Xp_l @ w
    return xa, xa[:, None] + np.sqrt(rho) * (Xp_l @ W)


def local_update_smw(xb_l, Xp_l, Y, d, g, rho):
    """The paper's local update in its SMW form, on inflated anomalies.

    Z = sqrt(rho) X'/sqrt(m-1); S_cz = Sigma^{-1/2} C Z; S_inov = Sigma^{-1/2} d;
    EVD of Id + S_cz^T S_cz = Q Gamma Q^T;
    x^ = x + Z S_cz^T (S_inov - S_cz Q Gamma^-1 Q^T S_cz^T S_inov);
    X = sqrt(m-1) Z Q Gamma^{-1/2} Q^T + x^ 1^T."""
    m = Xp_l.shape[1]
    sq = np.sqrt(g)
    Z = np.sqrt(rho) * Xp_l / np.sqrt(m - 1)
    Scz = sq[:, None] * (np.sqrt(rho) * Y / np.sqrt(m - 1))
    Sinov = sq * d
    gam, Q = np.linalg.eigh(np.eye(m) + Scz.T @ Scz)
    inner = Sinov - Scz @ (Q @ ((Q.T @ (Scz.T @ Sinov)) / gam))
    xhat = xb_l + Z @ (Scz.T @ inner)
    X = np.sqrt(m - 1) * Z @ ((Q / np.sqrt(gam)) @ Q.T) + xhat[:, None]
    return xhat, X


def local_mean_gain(xb_l, Xp_l, Y, d, g, rho):
    """The paper's local Kalman gain form: x^ = x + H~ (y - y_bar) with
    H~ = Z S^T (I - S Q Gamma^-1 Q^T S^T) Sigma^{-1/2} (inflated anomalies)."""
    m = Xp_l.shape[1]
    sq = np.sqrt(g)
    Z = np.sqrt(rho) * Xp_l / np.sqrt(m - 1)
    S = sq[:, None] * (np.sqrt(rho) * Y / np.sqrt(m - 1))
    gam, Q = np.linalg.eigh(np.eye(m) + S.T @ S)
    M = np.eye(S.shape[0]) - S @ ((Q / gam) @ Q.T) @ S.T
    H = Z @ S.T @ M @ np.diag(sq)
    return xb_l + H @ d


def local_mean_kalman(xb_l, Xp_l, Y, d, g, rho):
    """Per-domain Kalman update with the inflated sample covariance
    P = rho X' X'^T/(m-1), brute force through the p_l x p_l inverse
    (Sec. 2.2 update and gain equations restricted to the domain; slopes with
    g = 0 carry no information and are dropped)."""
    m = Xp_l.shape[1]
    keep = g > 0
    Yk, dk, gk = Y[keep], d[keep], g[keep]
    Pyy = rho * (Yk @ Yk.T) / (m - 1) + np.diag(1.0 / gk)
    Pxy = rho * (Xp_l @ Yk.T) / (m - 1)
    return xb_l + Pxy @ np.linalg.solve(Pyy, dk)


def local_inputs(geom, dom, Yp, d, r_diag, params: Params):
    """L1: local slope anomalies, innovation and weights of one domain."""
    f = geo.taper(dom, params.b, params.taper_c)
    g = f * f / (params.r_scale * np.asarray(r_diag, dtype=np.float64)[dom.obs])
    return Yp[dom.obs], d[dom.obs], g


def analysis(geom, doms, Xb, y, r_diag, params: Params, keep=None):
    """F2 + L1-L5 + G: the analysis ensemble from the forecast ensemble.

    `keep` (optional dict) receives per-domain intermediates for tests."""
    Xb = np.asarray(Xb, dtype=np.float64)
    xb, Xp = ensemble_stats(Xb)
    Yp = geo.apply_slopes(geom, Xp)
    d = np.asarray(y, dtype=np.float64) - geo.apply_slopes(geom, xb)
    Xa = np.empty_like(Xb)
    for k, dom in enumerate(doms):
        Y, dl, g = local_inputs(geom, dom, Yp, d, r_diag, params)
        w, W, A, lam = local_weights(Y, dl, g, params.rho)
        _, Xa[dom.owned] = local_update(xb[dom.owned], Xp[dom.owned], w, W, params.rho)
        if keep is not None:
            keep.setdefault("w", []).append(w)
            keep.setdefault("W", []).append(W)
            keep.setdefault("A", []).append(A)
            keep.setdefault("b", []).append(Y.T @ (g * dl))
    return Xa


def step(geom, doms, Xa_prev, V, y, r_diag, params: Params):
    """One frame: forecast, analysis and, when params.piston is set, the
    differential-piston removal (the `piston` module)."""
    Xa = analysis(geom, doms, forecast(Xa_prev, V, params.a), y, r_diag, params)
    if params.piston:
        from . import piston
        Xa = piston.remove(geom, doms, Xa, y)
    return Xa


def residual_variance(xa_mean: np.ndarray, truth: np.ndarray) -> float:
    """Spatial variance over the valid nodes of the analysis-mean error, mean
    removed (the residual-phase variance behind the coherent energy, Sec. 5)."""
    e = np.asarray(xa_mean, dtype=np.float64) - np.asarray(truth, dtype=np.float64)
    return float(np.mean((e - e.mean()) ** 2))


def run(geom, doms, V_seq, y_seq, r_diag, params: Params, Xa0=None, truth=None):
    """T frames from X_a = Xa0 (zero ensemble by default, Sec. 3.1).

    Returns the final analysis ensemble, the analysis means per frame and, when
    `truth` is given, the residual variance per frame."""
    T = len(y_seq)
    m = V_seq[0].shape[1]
    Xa = np.zeros((geom.n_nodes, m)) if Xa0 is None else np.array(Xa0, dtype=np.float64)
    means, res = [], []
    for k in range(T):
        Xa = step(geom, doms, Xa, V_seq[k], y_seq[k], r_diag, params)
        means.append(Xa.mean(axis=1))
        if truth is not None:
            res.append(residual_variance(means[-1], truth[k]))
    return Xa, np.array(means), np.array(res)
