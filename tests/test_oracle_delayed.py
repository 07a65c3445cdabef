"""Pins of the oracle's delayed state (Sec. 2.2: x_k = [phi_k; phi_{k-1};
u_{k-1}; u_{k-2}], y_k = D phi_{k-1} - D N u_{k-2} + w_k): the Kalman update
of the four-block state for both forms of the filter, the delay-free limit,
the DM term's sign, the piston reading in this state, and the loop it
closes."""
import numpy as np
import pytest

from oracle import delayed as DL
from oracle import geometry as geo
from oracle import kalman
from oracle import letkf as ol
from paper_1408_7069_amd import workload as wl


def _dense_D(G):
    return np.stack([geo.apply_slopes(G, e) for e in np.eye(G.n_nodes)], axis=1)


def _four_block(G, n, D, P_phi, x_phi, u1, u2):
    """Covariance, observation matrix and mean of [phi_k; phi_{k-1}; u_{k-1};
    u_{k-2}] with the voltages known (zero covariance), C = [0, D, 0, -D]."""
    Pf = np.zeros((4 * n, 4 * n))
    Pf[:2 * n, :2 * n] = P_phi
    C = np.hstack([np.zeros_like(D), D, np.zeros_like(D), -D])
    return Pf, C, np.concatenate([x_phi, u1, u2])


def _tiny(seed, m=60):
    G = geo.geometry_for(3, None)
    doms = geo.domains(G, 3, 0)
    assert len(doms) == 1
    rng = np.random.default_rng(seed)
    return G, doms, G.n_nodes, m, rng


@pytest.mark.parametrize("a,u_on", [(0.95, False), (0.95, True), (0.6, True)])
def test_literal_form_is_the_kalman_update_with_the_sample_covariance(a, u_on):
    # one domain over the whole pupil, full-rank ensemble: the two phase blocks
    # of the stacked ETKF are the Kalman update (Sec. 2.2) of the four-block
    # state with the sample covariance of the stacked forecast ensemble
    G, doms, n, m, rng = _tiny(3)
    prm = ol.Params(a=a, rho=1.0, b=3, h=0)
    Xa_prev = rng.standard_normal((n, m))
    V = 0.3 * rng.standard_normal((n, m))
    r = rng.uniform(0.05, 0.2, G.n_slopes)
    u1 = rng.standard_normal(n) if u_on else np.zeros(n)
    u2 = rng.standard_normal(n) if u_on else np.zeros(n)
    y = rng.standard_normal(G.n_slopes)
    Xu, Xl = DL.literal_analysis(G, doms, *DL.literal_forecast(Xa_prev, V, a), y, r, prm,
                                 u_prev2=u2 if u_on else None)
    Xb = np.vstack([a * Xa_prev + V, Xa_prev])
    xb = Xb.mean(axis=1)
    Zp = (Xb - xb[:, None]) / np.sqrt(m - 1)
    Pf, C, x0 = _four_block(G, n, _dense_D(G), Zp @ Zp.T, xb, u1, u2)
    xa, Pa, _ = kalman.kalman_update(x0, Pf, C, np.diag(r), y)
    assert np.allclose(Xu.mean(axis=1), xa[:n], atol=1e-10)
    assert np.allclose(Xl.mean(axis=1), xa[n:2 * n], atol=1e-10)
    assert np.allclose(xa[2 * n:], np.concatenate([u1, u2]))   # the voltages are not moved
    Za = np.vstack([Xu, Xl])
    Za = (Za - Za.mean(axis=1, keepdims=True)) / np.sqrt(m - 1)
    assert np.allclose(Za @ Za.T, Pa[:2 * n, :2 * n], atol=1e-10)


@pytest.mark.parametrize("a", [0.99, 0.7])
def test_structured_form_is_the_kalman_update_when_the_model_noise_is_independent(a):
    # prior of [phi_k; phi_{k-1}]: [[a^2 P + S_v, a P], [a P, P]] (phi_k =
    # a phi_{k-1} + v_k, v_k independent) with P the sample covariance of the
    # lower forecast; its Kalman update moves the lower block as the library
    # form does, and the upper block by a times that (the gain of the upper
    # block is a times the gain of the lower one)
    G, doms, n, m, rng = _tiny(4)
    prm = ol.Params(a=a, rho=1.0, b=3, h=0)
    Xa_prev = rng.standard_normal((n, m))
    V = 0.3 * rng.standard_normal((n, m))
    r = rng.uniform(0.05, 0.2, G.n_slopes)
    u1, u2 = rng.standard_normal(n), rng.standard_normal(n)
    y = rng.standard_normal(G.n_slopes)
    Xa = DL.step(G, doms, Xa_prev, V, y, r, prm, u_prev2=u2)
    Xb = a * Xa_prev + V
    xb = Xb.mean(axis=1)
    Zp = (Xb - xb[:, None]) / np.sqrt(m - 1)
    P = Zp @ Zp.T
    B = rng.standard_normal((n, n))
    Sv = B @ B.T                                               # any model-noise covariance
    Pphi = np.block([[a * a * P + Sv, a * P], [a * P, P]])
    vbar = rng.standard_normal(n)
    Pf, C, x0 = _four_block(G, n, _dense_D(G), Pphi, np.concatenate([a * xb + vbar, xb]), u1, u2)
    xa, Pa, _ = kalman.kalman_update(x0, Pf, C, np.diag(r), y)
    assert np.allclose(Xa.mean(axis=1), xa[n:2 * n], atol=1e-10)
    assert np.allclose(xa[:n], a * xa[n:2 * n] + vbar, atol=1e-10)
    Za = (Xa - Xa.mean(axis=1, keepdims=True)) / np.sqrt(m - 1)
    assert np.allclose(Za @ Za.T, Pa[n:2 * n, n:2 * n], atol=1e-10)


def test_without_model_noise_both_forms_are_the_delay_free_analysis():
    # a = 1 and V = 0: the stacked blocks coincide, and the literal form's two
    # blocks and the library form are all the delay-free analysis
    G = geo.geometry_for(12, 0.28)
    doms = geo.domains(G, 4, 1)
    rng = np.random.default_rng(5)
    prm = ol.Params(a=1.0, rho=1.05, b=4, h=1, taper_c=1.5)
    Xa_prev = rng.standard_normal((G.n_nodes, 24))
    Z = np.zeros_like(Xa_prev)
    r = np.full(G.n_slopes, 0.01)
    y = geo.apply_slopes(G, rng.standard_normal(G.n_nodes))
    Xu, Xl = DL.literal_analysis(G, doms, *DL.literal_forecast(Xa_prev, Z, 1.0), y, r, prm)
    ref = ol.analysis(G, doms, Xa_prev, y, r, prm)
    assert np.allclose(Xu, ref, atol=1e-12) and np.allclose(Xl, ref, atol=1e-12)
    assert np.allclose(DL.step(G, doms, Xa_prev, Z, y, r, prm), ref, atol=1e-12)


def test_dm_term_is_the_pseudo_open_loop_innovation():
    # y_bar = D x - D u_{k-2}: stepping with (y, u) equals stepping with the
    # pseudo-open-loop slopes y + D u and no command (pistons included)
    G = geo.geometry_for(10, 0.2)
    doms = geo.domains(G, 3, 1)
    rng = np.random.default_rng(7)
    prm = ol.Params(a=0.97, rho=1.02, b=3, h=1, piston=True)
    Xa = rng.standard_normal((G.n_nodes, 16))
    V = 0.2 * rng.standard_normal((G.n_nodes, 16))
    r = np.full(G.n_slopes, 0.02)
    u2 = rng.standard_normal(G.n_nodes)
    y = rng.standard_normal(G.n_slopes)
    a1 = DL.step(G, doms, Xa, V, y, r, prm, u_prev2=u2)
    a2 = DL.step(G, doms, Xa, V, y + geo.apply_slopes(G, u2), r, prm)
    assert np.allclose(a1, a2, atol=1e-11)
    l1 = DL.literal_step(G, doms, Xa, V, y, r, prm, u_prev2=u2)
    l2 = DL.literal_step(G, doms, Xa, V, y + geo.apply_slopes(G, u2), r, prm)
    assert np.allclose(l1[0], l2[0], atol=1e-11) and np.allclose(l1[1], l2[1], atol=1e-11)


@pytest.mark.parametrize("u_on", [False, True])
def test_planted_pistons_in_the_delayed_state(u_on):
    # the lower block explains the slopes up to per-domain constants; the fit
    # on x_a - u_{k-2} recovers them (up to their common mean)
    G = geo.geometry_for(12, 0.28)
    doms = geo.domains(G, 4, 1)
    own = geo.owner_map(G, doms)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(G.n_nodes)
    u2 = rng.standard_normal(G.n_nodes) if u_on else np.zeros(G.n_nodes)
    y = geo.apply_slopes(G, x - u2)
    p0 = rng.standard_normal(len(doms))
    A = rng.standard_normal((G.n_nodes, 6))
    A -= A.mean(axis=1, keepdims=True)
    Xl = (x + p0[own])[:, None] + A
    pi = DL.pistons(G, doms, Xl, y, u_prev2=u2 if u_on else None)
    assert np.allclose(pi, -(p0 - p0.mean()), atol=1e-10)


def test_command_is_the_two_step_prediction():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((30, 8))
    assert np.allclose(DL.command(X, 0.9), 0.81 * X.mean(axis=1))


def _loop_case(N=8, m=24, T=60, a=0.99, seed=11):
    G = geo.geometry_for(N, None)
    doms = geo.domains(G, 2, 1)
    rng = np.random.default_rng(seed)
    ij = G.node_coords()
    grid = wl.ar1_truth(N, T + 1, 0.4, 0.15, 25.0, a, rng)
    truth = np.array([g[ij[:, 0], ij[:, 1]] for g in grid])
    V = [np.sqrt(1 - a * a) * np.stack([s[ij[:, 0], ij[:, 1]]
                                        for s in wl.vk_screens(2 * (N + 1), 0.4, 0.15, 25.0, m, rng)], axis=1)
         for _ in range(T)]
    noise = [wl.gaussian_noise(G.n_slopes, 0.1, rng) for _ in range(T)]
    return G, doms, truth, V, noise, np.full(G.n_slopes, 0.01)


def test_the_loop_corrects_the_turbulence():
    # 8x8 pupil, m = 24, AR(1) truth with von Karman innovations: after the
    # first frames the residual phase under the commands is the two-frame
    # prediction error, a small fraction of the turbulence
    a = 0.99
    G, doms, truth, V, noise, r = _loop_case(a=a)
    prm = ol.Params(a=a, rho=1.05, b=2, h=1, piston=True)
    cmds, res, _ = DL.closed_loop(G, doms, truth, V, noise, r, prm)
    var = lambda v: float(np.mean((v - v.mean()) ** 2))
    late = range(30, len(res))
    res_v = np.mean([var(res[k]) for k in late])
    tur_v = np.mean([var(truth[k + 1]) for k in late])
    assert res_v < 0.1 * tur_v, (res_v, tur_v)
    assert np.allclose(res[5], truth[6] - cmds[4])     # residual = phi_k - u_{k-1}
