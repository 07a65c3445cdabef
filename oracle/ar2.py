"""Second-order autoregressive turbulence model (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's model is AR(1) (Sec. 2.2, A_tur); its conclusion (Sec. 6) names
the AR(2) model as the extension: phi_{k+1} = a1 phi_k + a2 phi_{k-1} + v_k.
Reading used here ("member history"): each member is forecast from its own
analyses of the last two frames,

    X_b(k+1) = a1 X_a(k) + a2 X_a(k-1) + V,

and only the current phase is analysed (the lagged block is not smoothed by
the new slopes; updating it through the ensemble cross-covariance brings the
sampling noise of the delayed-state form).  With a2 = 0 this is the AR(1)
frame.  For a stationary process of unit variance the innovation has standard
deviation sqrt((1 + a2) ((1 - a2)^2 - a1^2) / (1 - a2)), and the lag-1 and
lag-2 correlations are rho1 = a1 / (1 - a2), rho2 = a1 rho1 + a2
(Yule-Walker).
"""
from __future__ import annotations

import numpy as np

from . import letkf as ol


def forecast(Xa, Xa_prev, V, a1, a2):
    """X_b = a1 X_a(k) + a2 X_a(k-1) + V."""
    return (a1 * np.asarray(Xa, np.float64) + a2 * np.asarray(Xa_prev, np.float64)
            + np.asarray(V, np.float64))


def step(geom, doms, Xa, Xa_prev, V, y, r_diag, params, a2):
    """One frame with the AR(2) forecast (params.a is a1); pistons when on."""
    Xb = forecast(Xa, Xa_prev, V, params.a, a2)
    Xn = ol.analysis(geom, doms, Xb, y, r_diag, params)
    if params.piston:
        from . import piston
        Xn = piston.remove(geom, doms, Xn, y)
    return Xn


def yule_walker(rho1, rho2):
    """(a1, a2) of the AR(2) process with lag-1 and lag-2 correlations."""
    d = 1.0 - rho1 * rho1
    return rho1 * (1.0 - rho2) / d, (rho2 - rho1 * rho1) / d


def innovation_std(a1, a2):
    """Innovation standard deviation of a unit-variance stationary AR(2)."""
    return float(np.sqrt((1.0 + a2) * ((1.0 - a2) ** 2 - a1 * a1) / (1.0 - a2)))
