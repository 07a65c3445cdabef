"""Pins of the covariance-localisation variant (Sec. 4: the prior covariance
tapered by a Schur product): the local slope operator, the local analysis's
mean with the taper off, the dense Kalman update with the tapered covariance
on one domain, the deterministic-EnKF covariance identity, the rank the
taper adds, and the filter loop against the local analysis."""
import numpy as np
import pytest

from oracle import blend as BL
from oracle import cl as CL
from oracle import geometry as geo
from oracle import letkf as ol
from paper_1408_7069_amd import workload as wl


def _case(N, eps, m, seed):
    G = geo.geometry_for(N, eps)
    rng = np.random.default_rng(seed)
    Xb = rng.standard_normal((G.n_nodes, m)) + 2.0 * rng.standard_normal(G.n_nodes)[:, None]
    y = rng.standard_normal(G.n_slopes)
    r = rng.uniform(0.01, 0.04, G.n_slopes)
    return G, Xb, y, r


def test_local_slope_operator_is_the_dense_one():
    G, _, _, r = _case(12, 0.28, 4, 1)
    D = geo.slope_matrix(G)
    prm = ol.Params(b=4, h=1, r_scale=1.7)
    for dom in geo.domains(G, 4, 1):
        P, Dt = CL.local_operators(G, dom, r, prm)
        assert np.array_equal(P, BL.patch_nodes(G, dom))
        ref = D[np.ix_(dom.obs, P)] / np.sqrt(1.7 * r[dom.obs])[:, None]
        assert np.abs(Dt - ref).max() == 0.0
        # the patch holds every node the region's slopes see
        rest = np.setdiff1d(np.arange(G.n_nodes), P)
        assert np.abs(D[np.ix_(dom.obs, rest)]).max(initial=0.0) == 0.0


@pytest.mark.parametrize("N,eps,b,h,m", [(12, 0.28, 4, 1, 16), (10, None, 2, 1, 24), (8, None, 3, 0, 12)])
def test_untapered_mean_is_the_local_analysis_mean(N, eps, b, h, m):
    G, Xb, y, r = _case(N, eps, m, 2)
    doms = geo.domains(G, b, h)
    prm = ol.Params(b=b, h=h, rho=1.07, r_scale=1.3, taper_c=0.0)
    a = CL.analysis(G, doms, Xb, y, r, prm)
    ref = ol.analysis(G, doms, Xb, y, r, prm)
    assert np.abs(a.mean(1) - ref.mean(1)).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("c", [0.0, 1.5, 3.0])
def test_one_domain_is_the_dense_tapered_kalman_update(c):
    # one domain covering the pupil: the mean is x_b + K d and the anomalies
    # sqrt(rho) (X' - K H X' / 2) with K = P_loc H^T (H P_loc H^T + R)^{-1},
    # P_loc = rho_xx o (rho X' X'^T / (m - 1)) over all nodes
    G, Xb, y, r = _case(6, None, 10, 3)
    doms = geo.domains(G, 6, 0)
    rho, s = 1.05, 1.2
    prm = ol.Params(b=6, h=0, rho=rho, r_scale=s, taper_c=c)
    out = CL.analysis(G, doms, Xb, y, r, prm)
    xb, Xp = ol.ensemble_stats(Xb)
    H = geo.slope_matrix(G)
    pos = G.node_coords().astype(float)
    dist = np.sqrt(((pos[:, None] - pos[None]) ** 2).sum(-1))
    taper = geo.gaspari_cohn(dist / c) if c > 0 else np.ones_like(dist)
    Ploc = taper * (rho * Xp @ Xp.T / (Xb.shape[1] - 1))
    K = Ploc @ H.T @ np.linalg.inv(H @ Ploc @ H.T + s * np.diag(r))
    assert np.abs(out.mean(1) - (xb + K @ (y - H @ xb))).max() <= 1e-10 * np.abs(xb).max()
    Xa = out - out.mean(1)[:, None]
    assert np.abs(Xa - np.sqrt(rho) * (Xp - 0.5 * K @ H @ Xp)).max() <= 1e-10 * np.abs(Xp).max()


def test_deterministic_enkf_covariance_identity():
    # untapered, one domain: the analysis covariance of the returned members
    # is P - K H P + K H P H^T K^T / 4 (Sakov & Oke 2008), P the inflated prior
    G, Xb, y, r = _case(6, None, 12, 4)
    doms = geo.domains(G, 6, 0)
    rho = 1.1
    prm = ol.Params(b=6, h=0, rho=rho, r_scale=1.0, taper_c=0.0)
    out = CL.analysis(G, doms, Xb, y, r, prm)
    m = Xb.shape[1]
    _, Xp = ol.ensemble_stats(Xb)
    P = rho * Xp @ Xp.T / (m - 1)
    H = geo.slope_matrix(G)
    K = P @ H.T @ np.linalg.inv(H @ P @ H.T + np.diag(r))
    Xa = out - out.mean(1)[:, None]
    Pa = Xa @ Xa.T / (m - 1)
    ref = P - K @ H @ P + 0.25 * K @ H @ P @ H.T @ K.T
    assert np.abs(Pa - ref).max() <= 1e-10 * np.abs(P).max()


def test_taper_raises_the_rank_and_keeps_the_covariance_definite():
    G, Xb, _, _ = _case(12, 0.28, 8, 5)
    dom = geo.domains(G, 4, 1)[5]
    P = BL.patch_nodes(G, dom)
    _, Xp = ol.ensemble_stats(Xb)
    C = Xp[P] @ Xp[P].T
    T = CL.node_correlation(G, P, 2.0)
    assert np.allclose(np.diag(T), 1.0) and np.allclose(T, T.T)
    ij = G.node_coords()[P]
    far = np.sqrt(((ij[:, None] - ij[None]) ** 2).sum(-1)) >= 4.0
    assert np.all(T[far] == 0.0)
    lam_raw = np.linalg.eigvalsh(C)
    lam = np.linalg.eigvalsh(T * C)
    assert np.sum(lam_raw > 1e-9 * lam_raw.max()) <= 7          # rank m - 1
    assert lam.min() > 1e-9 * lam.max() and len(P) > 8          # full rank: definite


def test_cl_filter_loop_beats_the_local_analysis():
    # 12x12 square pupil, 4x4 domains, halo 1, m = 32, a = 0.99, pistons:
    # with a 3-pitch taper the residual variance is well below the local
    # analysis's; untapered it is close to it
    N, b, h, m, T, a = 12, 4, 1, 32, 120, 0.99
    G = geo.geometry_for(N, None)
    ij = G.node_coords()
    doms = geo.domains(G, b, h)
    rng = np.random.default_rng(5)
    truth = np.array([g[ij[:, 0], ij[:, 1]] for g in wl.ar1_truth(N, T, 0.4, 0.15, 25.0, a, rng)])
    r = np.full(G.n_slopes, 0.04)
    out = {}
    for name, c in (("la", 0.0), ("cl0", 0.0), ("cl3", 3.0)):
        rng = np.random.default_rng(9)
        prm = ol.Params(a=a, rho=1.05, b=b, h=h, piston=True, taper_c=c)
        Xa = np.zeros((G.n_nodes, m))
        err = []
        for k in range(T):
            V = np.sqrt(1 - a * a) * np.stack(
                [s[ij[:, 0], ij[:, 1]] for s in wl.vk_screens(2 * (N + 1), 0.4, 0.15, 25.0, m, rng)], 1)
            y = geo.apply_slopes(G, truth[k]) + 0.2 * rng.standard_normal(G.n_slopes)
            Xa = ol.step(G, doms, Xa, V, y, r, prm) if name == "la" else CL.step(G, doms, Xa, V, y, r, prm)
            err.append(ol.residual_variance(Xa.mean(1), truth[k]))
        out[name] = float(np.mean(err[T // 2:]))
    assert out["cl3"] < 0.7 * out["la"], out
    assert out["cl0"] < 1.3 * out["la"], out
