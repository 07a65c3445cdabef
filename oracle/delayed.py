"""The paper's state with the measurement delay and the DM terms (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 writes the AO state as x_k = [phi_k; phi_{k-1}; u_{k-1}; u_{k-2}]
with the AR(1) turbulence, the voltage shift register and the observation
y_k = D phi_{k-1} - D N u_{k-2} + w_k: the wavefront sensor reads, at frame k,
the residual of the phase of the previous frame under the command applied
then.  Only the two phase blocks are estimated (the voltages are known); with
A_1 = [[a I, 0], [I, 0]] and C_1 = [0, D].  The control part (Sec. 2.2) is the
least-squares projection of the predicted phase on the DM space,
u_k = P phi_hat_{k+1/k}.  Reading: a zonal DM whose actuators are the valid
phase nodes, N = P = I.

Two forms of the filter on this state are written out.

`literal_*`: the ETKF on the two stacked blocks as the equations read
(Sec. 3.1.2 prediction with A_1, Sec. 3.1.1 / 4.2 update with S_cz built from
the slopes of the lower block): upper members a X_a^up + V, lower members
X_a^up, and the same mean weights w and transform W move both blocks through
the ensemble's cross-covariance.  Pinned against the Kalman update of the
four-block state.  With m <= 64 and 4 x 4-subaperture domains it diverges on
the workloads here: phi_k = a phi_{k-1} + v_k with v_k independent of all
slopes up to y_k, but the sampled covariance of the fresh model-noise members
with the observed block (relative size sigma_v / (sqrt(m) sigma_a), sigma_a
the analysis spread) moves the upper block at random, and the error feeds back
through the next frame's lower block.

The form used by the library (`step`, `command`, `closed_loop`) keeps the
model's structure for the unobserved block, as the Kalman filter does: the
update of phi_k is a times the update of phi_{k-1} (the gain of the upper
block is a times the gain of the lower one when the model noise is independent
of the slopes), so only the lower block is analysed, by the local ETKF on the
slopes of y_k with y_bar = D x_b - D N u_{k-2}, and the ensemble carried to
the next frame is a X_a^low + V -- the forecast the delay-free frame forms.
The command is u_k = P phi_hat_{k+1/k} = a^2 x_a^low (the model noise taken
at its zero mean).  Reading for the piston step (Sec. 4.4) in this state: the
pistons are fitted to the slopes the lower block explains, on
x_a^low - N u_{k-2} against y_k.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from . import letkf as ol


# ---------------------------------------------------------------- literal form
def literal_forecast(Xa_up, V, a):
    """A_1 on the two blocks: (a X_a^up + V, X_a^up)."""
    Xa_up = np.asarray(Xa_up, np.float64)
    return a * Xa_up + np.asarray(V, np.float64), Xa_up.copy()


def literal_analysis(geom, doms, Xb_up, Xb_low, y, r_diag, params, u_prev2=None):
    """Local analyses of the two stacked blocks from the slopes of the lower
    one.  Returns (Xa_up, Xa_low)."""
    Xb_up = np.asarray(Xb_up, np.float64)
    Xb_low = np.asarray(Xb_low, np.float64)
    xu, Xpu = ol.ensemble_stats(Xb_up)
    xl, Xpl = ol.ensemble_stats(Xb_low)
    Yp = geo.apply_slopes(geom, Xpl)
    d = np.asarray(y, np.float64) - predicted_slopes(geom, xl, u_prev2)
    Xa_up, Xa_low = np.empty_like(Xb_up), np.empty_like(Xb_low)
    for dom in doms:
        Y, dl, g = ol.local_inputs(geom, dom, Yp, d, r_diag, params)
        w, W, _, _ = ol.local_weights(Y, dl, g, params.rho)
        o = dom.owned
        _, Xa_up[o] = ol.local_update(xu[o], Xpu[o], w, W, params.rho)
        _, Xa_low[o] = ol.local_update(xl[o], Xpl[o], w, W, params.rho)
    return Xa_up, Xa_low


def literal_step(geom, doms, Xa_up_prev, V, y, r_diag, params, u_prev2=None):
    """One frame of the stacked-block ETKF: (Xa_up, Xa_low); pistons (when
    on) fitted on the lower block and applied to both."""
    Xb_up, Xb_low = literal_forecast(Xa_up_prev, V, params.a)
    Xa_up, Xa_low = literal_analysis(geom, doms, Xb_up, Xb_low, y, r_diag, params, u_prev2)
    if params.piston:
        pi = pistons(geom, doms, Xa_low, y, u_prev2)
        own = geo.owner_map(geom, doms)
        Xa_up, Xa_low = Xa_up + pi[own][:, None], Xa_low + pi[own][:, None]
    return Xa_up, Xa_low


# --------------------------------------------------------- the library's form
def predicted_slopes(geom, x_mean, u_prev2=None):
    """y_bar = D x - D N u_{k-2} (N = I)."""
    ybar = geo.apply_slopes(geom, np.asarray(x_mean, np.float64))
    if u_prev2 is not None:
        ybar = ybar - geo.apply_slopes(geom, np.asarray(u_prev2, np.float64))
    return ybar


def pistons(geom, doms, Xa_low, y, u_prev2=None):
    """Sec. 4.4 pistons of the lower block, fitted on x_a^low - N u_{k-2}."""
    from . import piston
    xm = np.asarray(Xa_low, np.float64).mean(axis=1)
    if u_prev2 is not None:
        xm = xm - np.asarray(u_prev2, np.float64)
    return piston.pistons(geom, doms, xm, y)


def step(geom, doms, Xa_prev, V, y, r_diag, params, u_prev2=None):
    """One frame: the lower-block analysis X_a^low of phi_{k-1} from
    X_b = a X_a_prev + V (the previous frame's a X_a^low + V) and the slopes
    y_k with the DM term; pistons when on."""
    Xb = ol.forecast(Xa_prev, V, params.a)
    xb, Xp = ol.ensemble_stats(Xb)
    Yp = geo.apply_slopes(geom, Xp)
    d = np.asarray(y, np.float64) - predicted_slopes(geom, xb, u_prev2)
    Xa = np.empty_like(Xb)
    for dom in doms:
        Y, dl, g = ol.local_inputs(geom, dom, Yp, d, r_diag, params)
        w, W, _, _ = ol.local_weights(Y, dl, g, params.rho)
        _, Xa[dom.owned] = ol.local_update(xb[dom.owned], Xp[dom.owned], w, W, params.rho)
    if params.piston:
        pi = pistons(geom, doms, Xa, y, u_prev2)
        Xa = Xa + pi[geo.owner_map(geom, doms)][:, None]
    return Xa


def command(Xa_low, a):
    """u_k = P phi_hat_{k+1/k} = a^2 x_a^low (N = P = I)."""
    return a * a * np.asarray(Xa_low, np.float64).mean(axis=1)


def closed_loop(geom, doms, truth, V_seq, noise_seq, r_diag, params, Xa0=None):
    """The loop of Sec. 2.2 driven by a true phase sequence.

    truth[t] is phi_t for t = 0..T; at frame k = 1..T the sensor reads
    y_k = D (phi_{k-1} - u_{k-2}) + noise_seq[k-1], the filter steps with
    V_seq[k-1] and commands u_k; the residual during frame k is
    phi_k - u_{k-1} (commands before the first frame are zero).  Returns
    (commands u_1..u_T, residual phases of frames 1..T, analyses)."""
    n = geom.n_nodes
    m = V_seq[0].shape[1]
    Xa = np.zeros((n, m)) if Xa0 is None else np.asarray(Xa0, np.float64)
    u1, u2 = np.zeros(n), np.zeros(n)          # u_{k-1}, u_{k-2}
    cmds, res, ana = [], [], []
    for k in range(1, len(truth)):
        y = geo.apply_slopes(geom, truth[k - 1] - u2) + noise_seq[k - 1]
        Xa = step(geom, doms, Xa, V_seq[k - 1], y, r_diag, params, u_prev2=u2)
        res.append(truth[k] - u1)
        u = command(Xa, params.a)
        cmds.append(u)
        ana.append(Xa)
        u2, u1 = u1, u
    return np.array(cmds), np.array(res), ana
