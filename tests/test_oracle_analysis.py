"""Pins of the oracle's local ETKF analysis: the exact Kalman limit, agreement
of three independent update forms with a per-domain brute-force Kalman
update, and the invariants the symmetric square-root transform must keep."""
import numpy as np
import pytest

from oracle import geometry as geo
from oracle import kalman
from oracle import letkf as L


def _ensemble(n, m, rng, scale=1.0):
    X = scale * rng.standard_normal((n, m))
    return X


@pytest.mark.parametrize("m", [2, 3, 8, 40])
def test_exact_kalman_limit_one_domain(m):
    # one domain covering the pupil, no taper: the ensemble analysis mean and
    # covariance equal the Kalman update with the inflated sample covariance
    rng = np.random.default_rng(m)
    G = geo.Geometry(geo.square_mask(3))
    doms = geo.domains(G, 8, 0)
    assert len(doms) == 1
    n, p = G.n_nodes, G.n_slopes
    Xb = _ensemble(n, m, rng, 2.0)
    r = rng.uniform(0.05, 0.4, p)
    y = rng.standard_normal(p)
    for rho in (1.0, 1.3):
        prm = L.Params(rho=rho, b=8, h=0)
        Xa = L.analysis(G, doms, Xb, y, r, prm)
        xb, Xp = L.ensemble_stats(Xb)
        P = rho * Xp @ Xp.T / (m - 1)
        xa_kf, Pa_kf, _ = kalman.kalman_update(xb, P, geo.slope_matrix(G), np.diag(r), y)
        xa, Xap = L.ensemble_stats(Xa)
        assert np.allclose(xa, xa_kf, atol=1e-12 * (1 + np.abs(xa_kf).max()))
        assert np.allclose(Xap @ Xap.T / (m - 1), Pa_kf, atol=1e-12 * (1 + np.abs(Pa_kf).max()))


def _local_case(seed, m=12, taper_c=0.0, N=8, b=2, h=1):
    rng = np.random.default_rng(seed)
    G = geo.Geometry(geo.pupil_mask(N, 0.2) if N > 8 else geo.square_mask(N))
    doms = geo.domains(G, b, h)
    Xb = _ensemble(G.n_nodes, m, rng, 1.5)
    y = rng.standard_normal(G.n_slopes)
    r = rng.uniform(0.02, 0.2, G.n_slopes)
    prm = L.Params(rho=1.07, r_scale=1.3, b=b, h=h, taper_c=taper_c)
    return G, doms, Xb, y, r, prm


@pytest.mark.parametrize("taper_c", [0.0, 1.5])
def test_three_forms_and_local_kalman_agree(taper_c):
    G, doms, Xb, y, r, prm = _local_case(3, taper_c=taper_c)
    xb, Xp = L.ensemble_stats(Xb)
    Yp = geo.apply_slopes(G, Xp)
    d = y - geo.apply_slopes(G, xb)
    for dom in doms:
        Y, dl, g = L.local_inputs(G, dom, Yp, d, r, prm)
        w, W, A, lam = L.local_weights(Y, dl, g, prm.rho)
        xa, Xa = L.local_update(xb[dom.owned], Xp[dom.owned], w, W, prm.rho)
        xs, Xs = L.local_update_smw(xb[dom.owned], Xp[dom.owned], Y, dl, g, prm.rho)
        xg = L.local_mean_gain(xb[dom.owned], Xp[dom.owned], Y, dl, g, prm.rho)
        xk = L.local_mean_kalman(xb[dom.owned], Xp[dom.owned], Y, dl, g, prm.rho)
        sc = 1 + np.abs(xa).max()
        assert np.abs(xa - xs).max() < 1e-12 * sc
        assert np.abs(xa - xg).max() < 1e-12 * sc
        assert np.abs(xa - xk).max() < 1e-11 * sc
        assert np.abs(Xa - Xs).max() < 1e-12 * (1 + np.abs(Xa).max())


def test_transform_invariants():
    G, doms, Xb, y, r, prm = _local_case(5, m=16, taper_c=2.0, N=12, b=4, h=1)
    keep = {}
    Xa = L.analysis(G, doms, Xb, y, r, prm, keep=keep)
    m = Xb.shape[1]
    for W, A in zip(keep["W"], keep["A"]):
        assert np.abs(W - W.T).max() < 1e-13
        assert np.abs(W @ np.ones(m) - 1.0).max() < 1e-12
        # 1 is an eigenvector of A~ with eigenvalue (m-1)/rho
        assert np.abs(A @ np.ones(m) - (m - 1) / prm.rho).max() < 1e-9 * np.abs(A).max()
    # member mean of the analysis is the analysis mean: anomalies sum to zero
    xa_direct = np.empty(G.n_nodes)
    xb, Xp = L.ensemble_stats(Xb)
    for dom, w in zip(doms, keep["w"]):
        xa_direct[dom.owned] = xb[dom.owned] + Xp[dom.owned] @ w
    assert np.abs(Xa.mean(axis=1) - xa_direct).max() < 1e-12 * (1 + np.abs(xa_direct).max())


def test_zero_spread_keeps_forecast():
    G, doms, Xb, y, r, prm = _local_case(7)
    Xb = np.repeat(Xb[:, :1], Xb.shape[1], axis=1)
    Xa = L.analysis(G, doms, Xb, y, r, prm)
    assert np.array_equal(Xa, Xb)


def test_first_frame_from_zero_ensemble_is_the_noise():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((30, 5))
    assert np.array_equal(L.forecast(np.zeros((30, 5)), V, 0.99), V)


def test_inflation_and_noise_scale_equivalences():
    G, doms, Xb, y, r, prm = _local_case(11, taper_c=1.0)
    xb = Xb.mean(axis=1, keepdims=True)
    rho = prm.rho
    # rho with anomalies X' equals rho = 1 with anomalies sqrt(rho) X'
    Xa1 = L.analysis(G, doms, Xb, y, r, prm)
    prm1 = L.Params(rho=1.0, r_scale=prm.r_scale, b=prm.b, h=prm.h, taper_c=prm.taper_c)
    Xa2 = L.analysis(G, doms, xb + np.sqrt(rho) * (Xb - xb), y, r, prm1)
    assert np.abs(Xa1 - Xa2).max() < 1e-11 * (1 + np.abs(Xa1).max())
    # the noise scale s multiplies R: same as r -> s r with s = 1
    prm_s = L.Params(rho=rho, r_scale=1.0, b=prm.b, h=prm.h, taper_c=prm.taper_c)
    Xa3 = L.analysis(G, doms, Xb, y, prm.r_scale * r, prm_s)
    assert np.abs(Xa1 - Xa3).max() < 1e-12 * (1 + np.abs(Xa1).max())


def test_member_permutation_equivariance():
    G, doms, Xb, y, r, prm = _local_case(13)
    perm = np.random.default_rng(2).permutation(Xb.shape[1])
    Xa = L.analysis(G, doms, Xb, y, r, prm)
    Xp = L.analysis(G, doms, Xb[:, perm], y, r, prm)
    assert np.abs(Xa[:, perm] - Xp).max() < 1e-12 * (1 + np.abs(Xa).max())


def test_localisation_only_uses_the_observation_region():
    # changing slopes outside a domain's observation region leaves its owned
    # rows unchanged
    G, doms, Xb, y, r, prm = _local_case(17, N=12, b=4, h=1)
    Xa = L.analysis(G, doms, Xb, y, r, prm)
    dom = doms[0]
    outside = np.setdiff1d(np.arange(G.n_slopes), dom.obs)
    y2 = y.copy()
    y2[outside] += 5.0
    Xa2 = L.analysis(G, doms, Xb, y2, r, prm)
    assert np.array_equal(Xa[dom.owned], Xa2[dom.owned])
    assert not np.array_equal(Xa, Xa2)


def test_taper_scales_the_inverse_noise_std():
    # multiplying Sigma_w^{-1/2} by f is the same as dividing the noise
    # variance by f^2 (slopes with f = 0 then carry no information)
    G, doms, Xb, y, r, prm = _local_case(19, N=12, b=4, h=1, taper_c=1.2)
    xb, Xp = L.ensemble_stats(Xb)
    Yp = geo.apply_slopes(G, Xp)
    d = y - geo.apply_slopes(G, xb)
    for dom in doms:
        f = geo.taper(dom, prm.b, prm.taper_c)
        Y, dl, g = L.local_inputs(G, dom, Yp, d, r, prm)
        xa = L.local_mean_kalman(xb[dom.owned], Xp[dom.owned], Y, dl, g, prm.rho)
        keep = f > 0
        m = Xb.shape[1]
        Rl = prm.r_scale * r[dom.obs][keep] / f[keep] ** 2
        Yk, dk = Y[keep], dl[keep]
        K = prm.rho * Xp[dom.owned] @ Yk.T @ np.linalg.inv(prm.rho * Yk @ Yk.T + (m - 1) * np.diag(Rl))
        assert np.abs(xa - (xb[dom.owned] + K @ dk)).max() < 1e-11 * (1 + np.abs(xa).max())
