"""Pins of the online AR(1) refit (Sec. 4.2: the AR model updated during
the prediction step by an identification procedure): exact recovery on a
noise-free sequence, the least-squares estimate within its sampling error,
tracking of a change under forgetting, the clip, piston invariance, and the
model-noise scale."""
import numpy as np
import pytest

from oracle.refit import ArRefit


def _white_ar1(a, T, n, rng, x0=None):
    # spatially independent AR(1) nodes with unit stationary variance
    x = rng.standard_normal(n) if x0 is None else x0
    out = [x]
    for _ in range(T):
        x = a * x + np.sqrt(1 - a * a) * rng.standard_normal(n)
        out.append(x)
    return np.array(out)


def test_noise_free_sequence_gives_the_coefficient_exactly():
    x = [np.random.default_rng(0).standard_normal(50)]
    for _ in range(5):
        x.append(0.83 * x[-1])
    r = ArRefit(0.5, 0.9)
    for k in range(1, len(x)):
        r.update(x[k], x[k - 1])
        assert r.a == pytest.approx(0.83, abs=1e-13)


def test_least_squares_estimate_within_its_sampling_error():
    # n T pairs: the lag-1 least-squares estimate has standard deviation
    # sqrt((1 - a^2) / (n T))
    a, n, T = 0.95, 2000, 100
    x = _white_ar1(a, T, n, np.random.default_rng(1))
    r = ArRefit(0.5, 1.0)
    for k in range(1, len(x)):
        r.update(x[k], x[k - 1])
    assert abs(r.a - a) <= 4 * np.sqrt((1 - a * a) / (n * T))


def test_forgetting_follows_a_change_and_no_forgetting_does_not():
    rng = np.random.default_rng(2)
    x1 = _white_ar1(0.90, 200, 2000, rng)
    x2 = _white_ar1(0.99, 400, 2000, rng, x0=x1[-1])
    rf, r1 = ArRefit(0.5, 0.97), ArRefit(0.5, 1.0)
    for x in (x1, x2):
        for k in range(1, len(x)):
            rf.update(x[k], x[k - 1])
            r1.update(x[k], x[k - 1])
        if x is x1:
            assert rf.a == pytest.approx(0.90, abs=0.01)
    assert rf.a == pytest.approx(0.99, abs=0.003)
    assert 0.93 < r1.a < 0.98           # the whole history: between the two


def test_clip_to_the_stationary_range():
    x = [np.random.default_rng(3).standard_normal(20)]
    for g in (-0.7, -0.7):
        x.append(g * x[-1])
    r = ArRefit(0.5, 1.0)
    r.update(x[1], x[0])
    assert r.a == 0.0
    y = [x[0], 1.2 * x[0]]
    r = ArRefit(0.5, 1.0, a_max=0.999)
    r.update(y[1], y[0])
    assert r.a == 0.999


def test_piston_does_not_enter():
    x = _white_ar1(0.9, 50, 300, np.random.default_rng(4))
    r1, r2 = ArRefit(0.9, 0.98), ArRefit(0.9, 0.98)
    for k in range(1, len(x)):
        r1.update(x[k], x[k - 1])
        r2.update(x[k] + 3.0 * k, x[k - 1] + 3.0 * (k - 1))
    assert r1.a == pytest.approx(r2.a, abs=1e-12)


def test_noise_scale_keeps_the_stationary_variance():
    # Sigma_v = (1 - a^2) C: a bank drawn for a_0 is scaled so that the
    # stationary variance of x = a x + s v stays at C
    assert ArRefit(0.9, 0.98).noise_scale() == pytest.approx(1.0)
    r = ArRefit(0.6, 1.0)
    r.a = 0.8
    s = r.noise_scale()
    q0 = 1 - 0.6 ** 2                     # bank variance for a_0
    assert (s * s * q0) / (1 - 0.8 ** 2) == pytest.approx(1.0)


@pytest.mark.parametrize("a_true,a0,gain", [(0.99, 0.9, 1.15), (0.9, 0.99, 0.6)])
def test_refit_in_the_filter_loop_moves_toward_the_truth(a_true, a0, gain):
    # 8x8 pupil, 2x2 domains with halo 1, m = 32, pistons: the filter starts
    # from a mismatched a_0 (model noise drawn for a_0); the refit moves a
    # toward the true coefficient (Sec. 4.2: the model follows the
    # turbulence).  An a_0 above the truth trusts a stale forecast: the refit
    # removes most of that loss; one below it costs little, and the refit
    # stays within sampling noise of the fixed model
    from oracle import geometry as geo
    from oracle import letkf as ol
    from oracle import refit as RF
    from paper_1408_7069_amd import workload as wl
    N, m, T = 8, 32, 160
    G = geo.geometry_for(N, None)
    ij = G.node_coords()
    doms = geo.domains(G, 2, 1)
    rng = np.random.default_rng(5)
    truth = np.array([g[ij[:, 0], ij[:, 1]] for g in wl.ar1_truth(N, T, 0.4, 0.15, 25.0, a_true, rng)])
    sig = 0.2
    r = np.full(G.n_slopes, sig * sig)
    prm = ol.Params(a=a0, rho=1.05, b=2, h=1, piston=True)
    out = {}
    for refit in (False, True):
        rng = np.random.default_rng(9)
        Xa = np.zeros((G.n_nodes, m))
        rf = RF.ArRefit(a0, 0.98)
        err = []
        for k in range(T):
            V = np.sqrt(1 - a0 * a0) * np.stack(
                [s[ij[:, 0], ij[:, 1]] for s in wl.vk_screens(2 * (N + 1), 0.4, 0.15, 25.0, m, rng)], 1)
            y = geo.apply_slopes(G, truth[k]) + rng.standard_normal(G.n_slopes) * sig
            if refit:
                Xa, _ = RF.frame(G, doms, Xa, V, y, r, prm, rf)
            else:
                Xa = ol.step(G, doms, Xa, V, y, r, prm)
            err.append(ol.residual_variance(Xa.mean(1), truth[k]))
        out[refit] = (np.mean(err[50:]), rf.a)
    assert abs(out[True][1] - a_true) < 0.5 * abs(a0 - a_true), out
    assert out[True][0] < gain * out[False][0], out
