"""Reverse-mode gradient of the tuning loss of the local ETKF (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The loss is the residual-phase variance of the analysis mean, averaged over T
frames:

    J(rho, s, c) = (1/T) sum_k  mean_i ((e_k - mean(e_k))_i^2),
    e_k = x_a,k - phi_k   (analysis mean minus the true phase at the nodes),

the piston-removed error variance behind the coherent energy the paper uses as
its figure of merit (Sec. 5).  Its parameters are the three knobs of the
frame: the multiplicative inflation rho, the scale s of the noise covariance
(Sigma_w = s diag(r), Sec. 3.1.1) and the half width c of the Gaspari-Cohn
taper of the localisation (Sec. 4.1).  The noise draws V_k and the slopes y_k
are inputs, so J is a plain function of (rho, s, c).

`loss_and_grad` runs the frames forward (the `letkf` module's steps F1, F2,
L1-L5, G), keeps every analysis ensemble and then walks back through them.
The reverse of one frame, for the incoming adjoint Xa_bar of its analysis
ensemble (the loss term plus what the next forecast sends back):

  G / L5   per domain, owned rows:  xa_bar = Xa_bar 1,
           X'_bar += sqrt(rho) Xa_bar W + xa_bar w^T,  xb_bar += xa_bar,
           W_bar = sqrt(rho) X'^T Xa_bar,  w_bar = X'^T xa_bar,
           rho_bar += <Xa_bar, X' W> / (2 sqrt(rho));
  L4       w = A~^{-1} b:   b_bar = A~^{-1} w_bar,  A_bar -= b_bar w^T;
           W = sqrt(k) A~^{-1/2} with k = (m-1)/rho:
           k_bar += <W_bar, W> / (2k),
           A_bar += sqrt(k) Q (F o (Q^T sym(W_bar) Q)) Q^T, the adjoint of the
           matrix function through its eigendecomposition (Daleckii-Krein):
           F_ij = (f(l_i) - f(l_j)) / (l_i - l_j) for f(l) = l^{-1/2}, which is
           -1 / (s_i s_j (s_i + s_j)) with s = sqrt(l) (also the limit f'(l)
           on the diagonal and in degenerate clusters, no cancellation);
  L2       A~ = k I + Yt^T Yt, b = Yt^T dt with Yt = sqrt(g) Y, dt = sqrt(g) d:
           S = sym(A_bar),  k_bar += tr S,
           Yt_bar = 2 Yt S + dt b_bar^T,  dt_bar = Yt b_bar,
           sqrt(g)_bar_i = Yt_bar_i . Y_i + dt_bar_i d_i;
  L1       sqrt(g) = f(c) / sqrt(s r):  s_bar += -sqrt(g)_bar sqrt(g) / (2 s),
           c_bar += sqrt(g)_bar (df/dc) / sqrt(s r),
           df/dc = -GC'(dist / c) dist / c^2;
           Y_bar = sqrt(g) Yt_bar and d_bar = sqrt(g) dt_bar are added into the
           global slope-space adjoints at the domain's slopes (halo slopes
           receive from every domain that observes them);
  k        rho_bar += -k_bar (m-1) / rho^2;
  F2       X'_bar += D^T Y'_bar,  xb_bar -= D^T d_bar,
           Xb_bar = X'_bar - (X'_bar 1 / m) 1^T + xb_bar 1^T / m;
  F1       the previous analysis ensemble receives a Xb_bar.
With the differential-piston removal switched on, its adjoint (`piston`
module) is applied to Xa_bar first.

A domain whose forward analysis failed would keep its forecast; the oracle
has no such failure path (LAPACK eigh), so none is modelled here.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from . import letkf as lk
from . import piston


def loss(geom, doms, Xa0, V_seq, y_seq, truth, r_diag, params: lk.Params) -> float:
    """J for the frames of V_seq / y_seq from the analysis ensemble Xa0."""
    Xa = np.array(Xa0, dtype=np.float64)
    T = len(y_seq)
    tot = 0.0
    for k in range(T):
        Xa = lk.step(geom, doms, Xa, V_seq[k], y_seq[k], r_diag, params)
        tot += lk.residual_variance(Xa.mean(axis=1), truth[k])
    return tot / T


def _sym(M):
    return 0.5 * (M + M.T)


def _taper_dc(dom, b: int, c: float) -> np.ndarray:
    """d f / d c per local slope (zero when the taper is off)."""
    if c <= 0.0:
        return np.zeros(dom.obs.shape[0])
    dist = geo.taper_dist(dom, b)
    z = dist / c
    return -geo.gaspari_cohn_deriv(z) * dist / (c * c)


def frame_adjoint(geom, doms, Xa_prev, V, y, r_diag, params: lk.Params, Xa_bar):
    """Reverse of one frame: returns (a Xb_bar, (rho_bar, s_bar, c_bar)) for the
    adjoint Xa_bar of this frame's analysis ensemble."""
    p = params
    if p.piston:  # the piston removal came last in the frame
        Xa_bar = piston.remove_adjoint(geom, doms, Xa_bar)
    r_diag = np.asarray(r_diag, dtype=np.float64)
    Xb = lk.forecast(Xa_prev, V, p.a)
    n, m = Xb.shape
    xb, Xp = lk.ensemble_stats(Xb)
    Yp = geo.apply_slopes(geom, Xp)
    d = np.asarray(y, dtype=np.float64) - geo.apply_slopes(geom, xb)
    k = (m - 1) / p.rho
    Xp_bar = np.zeros((n, m))
    xb_bar = np.zeros(n)
    Yp_bar = np.zeros_like(Yp)
    d_bar = np.zeros_like(d)
    rho_bar = s_bar = c_bar = 0.0
    k_bar = 0.0
    for dom in doms:
        own = dom.owned
        Y, dl, g = lk.local_inputs(geom, dom, Yp, d, r_diag, p)
        sg = np.sqrt(g)
        Yt, dt = sg[:, None] * Y, sg * dl
        A = k * np.eye(m) + Yt.T @ Yt
        lam, Q = np.linalg.eigh(A)
        b = Yt.T @ dt
        w = Q @ ((Q.T @ b) / lam)
        W = np.sqrt(k) * (Q / np.sqrt(lam)) @ Q.T
        Xo = Xp[own]
        Xab = Xa_bar[own]
        # G / L5
        xa_bar = Xab.sum(axis=1)
        Xp_bar[own] += np.sqrt(p.rho) * Xab @ W + np.outer(xa_bar, w)
        xb_bar[own] += xa_bar
        W_bar = np.sqrt(p.rho) * Xo.T @ Xab
        w_bar = Xo.T @ xa_bar
        rho_bar += np.sum(Xab * (Xo @ W)) / (2.0 * np.sqrt(p.rho))
        # L4
        b_bar = Q @ ((Q.T @ w_bar) / lam)
        A_bar = -np.outer(b_bar, w)
        k_bar += np.sum(W_bar * W) / (2.0 * k)
        s_ = np.sqrt(lam)
        F = -1.0 / (np.outer(s_, s_) * (s_[:, None] + s_[None, :]))
        A_bar += np.sqrt(k) * Q @ (F * (Q.T @ _sym(W_bar) @ Q)) @ Q.T
        # L2
        S = _sym(A_bar)
        k_bar += np.trace(S)
        Yt_bar = 2.0 * Yt @ S + np.outer(dt, b_bar)
        dt_bar = Yt @ b_bar
        sg_bar = np.sum(Yt_bar * Y, axis=1) + dt_bar * dl
        # L1
        rs = np.sqrt(p.r_scale * r_diag[dom.obs])
        s_bar += -np.sum(sg_bar * sg) / (2.0 * p.r_scale)
        c_bar += np.sum(sg_bar * _taper_dc(dom, p.b, p.taper_c) / rs)
        np.add.at(Yp_bar, dom.obs, sg[:, None] * Yt_bar)
        np.add.at(d_bar, dom.obs, sg * dt_bar)
    rho_bar += -k_bar * (m - 1) / p.rho ** 2
    # F2
    Xp_bar += geo.apply_slopes_adjoint(geom, Yp_bar)
    xb_bar -= geo.apply_slopes_adjoint(geom, d_bar)
    Xb_bar = Xp_bar - Xp_bar.mean(axis=1, keepdims=True) + xb_bar[:, None] / m
    return p.a * Xb_bar, np.array([rho_bar, s_bar, c_bar])


def loss_adjoint(xa_mean, truth, weight: float, m: int) -> np.ndarray:
    """Adjoint of weight * residual_variance(X_a 1 / m, truth) with respect to
    the analysis ensemble X_a (every member gets 1/m of the mean's)."""
    e = np.asarray(xa_mean, dtype=np.float64) - np.asarray(truth, dtype=np.float64)
    g = weight * 2.0 * (e - e.mean()) / e.shape[0]
    return np.repeat(g[:, None] / m, m, axis=1)


def loss_and_grad(geom, doms, Xa0, V_seq, y_seq, truth, r_diag, params: lk.Params):
    """(J, dJ/d(rho, s, c)) by the forward frames and the reverse sweep."""
    T = len(y_seq)
    Xa = [np.array(Xa0, dtype=np.float64)]
    tot = 0.0
    for k in range(T):
        Xa.append(lk.step(geom, doms, Xa[-1], V_seq[k], y_seq[k], r_diag, params))
        tot += lk.residual_variance(Xa[-1].mean(axis=1), truth[k])
    m = Xa[0].shape[1]
    carry = np.zeros_like(Xa[0])
    grad = np.zeros(3)
    for k in range(T - 1, -1, -1):
        Xa_bar = carry + loss_adjoint(Xa[k + 1].mean(axis=1), truth[k], 1.0 / T, m)
        carry, gk = frame_adjoint(geom, doms, Xa[k], V_seq[k], y_seq[k], r_diag, params, Xa_bar)
        grad += gk
    return tot / T, grad


def central_difference(geom, doms, Xa0, V_seq, y_seq, truth, r_diag, params: lk.Params,
                       h: float = 1e-4) -> np.ndarray:
    """(J(t + h t) - J(t - h t)) / (2 h t) for each of rho, s, c (relative step)."""
    out = np.zeros(3)
    for i, name in enumerate(("rho", "r_scale", "taper_c")):
        t0 = getattr(params, name)
        step = h * t0
        vals = []
        for sgn in (1.0, -1.0):
            q = lk.Params(**{**params.__dict__, name: t0 + sgn * step})
            vals.append(loss(geom, doms, Xa0, V_seq, y_seq, truth, r_diag, q))
        out[i] = (vals[0] - vals[1]) / (2.0 * step)
    return out


__all__ = ["loss", "frame_adjoint", "loss_adjoint", "loss_and_grad", "central_difference"]
