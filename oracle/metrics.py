"""The paper's comparison criterion (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 5: the coherent energy E_coh = exp(-mean_k sigma^2_res(k)), with
sigma^2_res(k) the spatial variance of the residual phase at frame k and the
mean taken over time, and the loss of a control law against the KF,
loss = (E_coh^KF - E_coh) / E_coh^KF x 100 (%).
"""
from __future__ import annotations

import numpy as np


def spatial_variance(phase) -> float:
    """Variance over the valid nodes (mean removed) of one phase map."""
    p = np.asarray(phase, np.float64)
    return float(np.mean((p - p.mean()) ** 2))


def coherent_energy(residuals) -> float:
    """E_coh of a sequence of residual phases (already past the transient)."""
    return float(np.exp(-np.mean([spatial_variance(r) for r in residuals])))


def loss(e_kf: float, e: float) -> float:
    """Coherent-energy loss against the KF, in %."""
    return (e_kf - e) / e_kf * 100.0
