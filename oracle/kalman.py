"""The Kalman filter (oracle side): the brute-force update, the exact limit
the ensemble transform must reproduce when localisation is off, and the
stationary filter that the paper compares against.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2: update estimate x_a = x_b + H (y - C x_b), update covariance
(Id - H C) P, gain H = P C^T (C P C^T + Sigma_w)^{-1}, written with the full
p x p inverse; the asymptotic gain from the DARE of the prediction covariance.
Used only on small grids.
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


def dare(A: np.ndarray, C: np.ndarray, Q: np.ndarray, R: np.ndarray, tol: float = 1e-13,
         max_it: int = 60):
    """Asymptotic prediction covariance and Kalman gain of the stationary
    model x' = A x + v, y = C x + w (Sec. 2.2: the DARE of the prediction
    covariance, H = Sigma C^T (C Sigma C^T + Sigma_w)^{-1}).

    Solved by the structure-preserving doubling algorithm (Chu, Fan & Lin,
    2005) on the equivalent control-form equation with (A^T, C^T): A_0 = A^T,
    G_0 = C^T R^{-1} C, H_0 = Q;  W = I + G_k H_k,
    A_{k+1} = A_k W^{-1} A_k,  G_{k+1} = G_k + A_k W^{-1} G_k A_k^T,
    H_{k+1} = H_k + A_k^T H_k W^{-1} A_k  ->  H_k -> Sigma (quadratically).
    Returns (Sigma, H)."""
    n = A.shape[0]
    Ak = A.T.copy()
    Gk = C.T @ np.linalg.solve(R, C)
    Hk = Q.copy()
    for _ in range(max_it):
        W = np.eye(n) + Gk @ Hk
        WA = np.linalg.solve(W, Ak)
        WG = np.linalg.solve(W, Gk)
        A1 = Ak @ WA
        G1 = Gk + Ak @ WG @ Ak.T
        H1 = Hk + Ak.T @ Hk @ WA
        done = np.abs(H1 - Hk).max() <= tol * max(np.abs(H1).max(), 1.0)
        Ak, Gk, Hk = A1, 0.5 * (G1 + G1.T), 0.5 * (H1 + H1.T)
        if done:
            break
    S = Hk
    H = S @ C.T @ np.linalg.inv(C @ S @ C.T + R)
    return S, H


def closed_loop(D: np.ndarray, truth: np.ndarray, noise_seq, Sigma_v: np.ndarray, r_diag,
                a: float):
    """The optimal reference of Sec. 2.2: the stationary KF on the state
    [phi_k; phi_{k-1}] (A_1 = [[a I, 0], [I, 0]], C_1 = [0, D], Sigma_v on the
    first block) with the known voltages (y_bar = C_1 x - D u_{k-2}) and the
    command u_k = upper part of x_{k+1/k} (zonal DM, N = P = I).

    truth[t] = phi_t (t = 0..T) on the nodes; frame k reads
    y_k = D (phi_{k-1} - u_{k-2}) + noise_seq[k-1].  Returns (commands,
    residual phases phi_k - u_{k-1} of frames 1..T)."""
    n = D.shape[1]
    Z = np.zeros((n, n))
    A1 = np.block([[a * np.eye(n), Z], [np.eye(n), Z]])
    C1 = np.hstack([np.zeros_like(D), D])
    Q = np.block([[Sigma_v, Z], [Z, Z]])
    _, H = dare(A1, C1, Q, np.diag(np.asarray(r_diag, np.float64)))
    x = np.zeros(2 * n)
    u1, u2 = np.zeros(n), np.zeros(n)
    cmds, res = [], []
    for k in range(1, len(truth)):
        y = D @ (truth[k - 1] - u2) + noise_seq[k - 1]
        xu = x + H @ (y - (C1 @ x - D @ u2))
        res.append(truth[k] - u1)
        x = A1 @ xu
        u = x[:n].copy()
        cmds.append(u)
        u2, u1 = u1, u
    return np.array(cmds), np.array(res)
