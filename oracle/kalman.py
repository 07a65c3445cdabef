"""Brute-force Kalman update (oracle side), the exact limit the ensemble
transform must reproduce when localisation is off.

Sec. 2.2: update estimate x_a = x_b + H (y - C x_b), update covariance
(Id - H C) P, gain H = P C^T (C P C^T + Sigma_w)^{-1}, written with the full
p x p inverse.  Used only on tiny grids.
"""
from __future__ import annotations

import numpy as np


def kalman_update(xb: np.ndarray, P: np.ndarray, C: np.ndarray, R: np.ndarray,
                  y: np.ndarray):
    """Return (x_a, P_a, gain)."""
    S = C @ P @ C.T + R
    K = P @ C.T @ np.linalg.inv(S)
    xa = xb + K @ (y - C @ xb)
    Pa = (np.eye(P.shape[0]) - K @ C) @ P
    return xa, Pa, K
