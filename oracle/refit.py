"""Online refit of the AR(1) turbulence model (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 4.2 notes that the local gains need no DARE, so the filter can follow a
non-stationary turbulence, and that the AR model (A_1 and Sigma_v) can be
updated during the prediction step by an identification procedure it leaves
to be defined.  Reading used here: per instance, the least-squares lag-1
coefficient of the analysis means with exponential forgetting,

    S01_k = f S01_{k-1} + sum_n (x_k(n) - <x_k>) (x_{k-1}(n) - <x_{k-1}>)
    S11_k = f S11_{k-1} + sum_n (x_{k-1}(n) - <x_{k-1}>)^2
    a_k   = clip(S01_k / S11_k, 0, a_max)

(<.> the mean over the valid nodes: the piston is not observable), and the
model noise follows it, Sigma_v = (1 - a^2) C, i.e. a bank drawn for a_0 is
scaled by sqrt((1 - a_k^2) / (1 - a_0^2)).  The new coefficient is used from
the next frame on.
"""
from __future__ import annotations

import numpy as np


class ArRefit:
    def __init__(self, a0: float, forgetting: float, a_max: float = 0.9999):
        self.a0, self.f, self.a_max = float(a0), float(forgetting), float(a_max)
        self.s01 = self.s11 = 0.0
        self.a = float(a0)

    def update(self, x_now, x_prev) -> float:
        """Fold one frame's pair of analysis means in; returns the new a."""
        xn = np.asarray(x_now, np.float64)
        xp = np.asarray(x_prev, np.float64)
        xn = xn - xn.mean()
        xp = xp - xp.mean()
        self.s01 = self.f * self.s01 + float(xn @ xp)
        self.s11 = self.f * self.s11 + float(xp @ xp)
        if self.s11 > 0.0:
            self.a = float(np.clip(self.s01 / self.s11, 0.0, self.a_max))
        return self.a

    def noise_scale(self) -> float:
        """Factor on model noise drawn for a_0."""
        return float(np.sqrt((1.0 - self.a * self.a) / (1.0 - self.a0 * self.a0)))


def frame(geom, doms, Xa_prev, V, y, r_diag, params, refit: ArRefit, u_prev2=None):
    """One frame with the refitted model: the forecast uses the current a and
    the model noise V (drawn for a_0) scaled by noise_scale(); then the pair
    of analysis means (X_a(k), X_a(k-1)) updates the refit.  u_prev2 given:
    the closed-loop frame (delayed slopes and DM term), else the delay-free
    one.  Returns (X_a, the a this frame used)."""
    from dataclasses import replace
    from . import delayed as DL
    from . import letkf as ol
    a = refit.a
    p = replace(params, a=a)
    Vs = refit.noise_scale() * np.asarray(V, np.float64)
    Xa_prev = np.asarray(Xa_prev, np.float64)
    if u_prev2 is None:
        Xa = ol.step(geom, doms, Xa_prev, Vs, y, r_diag, p)
    else:
        Xa = DL.step(geom, doms, Xa_prev, Vs, y, r_diag, p, u_prev2=u_prev2)
    refit.update(Xa.mean(axis=1), Xa_prev.mean(axis=1))
    return Xa, a
