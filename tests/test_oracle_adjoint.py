"""Pins of the oracle's hand-written reverse-mode gradient: central finite
differences of the loss itself (second-order agreement), the transposed
state-to-state Jacobian by a directional-derivative test, and the closed form
of the eigendecomposition adjoint on a matrix with a degenerate cluster."""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import geometry as geo
from oracle import letkf as L


def _case(seed, N=8, m=12, T=5, taper_c=1.7, obscured=False, b=2, h=1):
    rng = np.random.default_rng(seed)
    G = geo.Geometry(geo.pupil_mask(N, 0.25) if obscured else geo.square_mask(N))
    doms = geo.domains(G, b, h)
    n, p = G.n_nodes, G.n_slopes
    truth = np.cumsum(rng.standard_normal((T, n)) * 0.3, axis=0)
    D = geo.slope_matrix(G)
    y = [D @ truth[k] + 0.1 * rng.standard_normal(p) for k in range(T)]
    V = [0.3 * rng.standard_normal((n, m)) for _ in range(T)]
    r = rng.uniform(0.005, 0.02, p)
    prm = L.Params(a=0.97, rho=1.1, r_scale=1.2, b=b, h=h, taper_c=taper_c)
    Xa0 = 0.2 * rng.standard_normal((n, m))
    return G, doms, Xa0, V, y, truth, r, prm


@pytest.mark.parametrize("seed,obscured,taper_c", [(5, False, 1.7), (6, True, 2.5), (7, False, 4.0)])
def test_gradient_matches_central_differences(seed, obscured, taper_c):
    args = _case(seed, N=10 if obscured else 8, obscured=obscured, taper_c=taper_c)
    J, g = AD.loss_and_grad(*args)
    assert J == pytest.approx(AD.loss(*args), rel=1e-14)
    fd = AD.central_difference(*args, h=1e-5)
    assert np.all(np.abs(fd - g) <= 1e-6 * np.abs(g) + 1e-12), (g, fd)


def test_finite_difference_error_is_second_order():
    # a reverse sweep with a wrong term would agree to first order at best;
    # the true gradient makes the central difference error fall as h^2
    args = _case(11)
    _, g = AD.loss_and_grad(*args)
    e3 = np.abs(AD.central_difference(*args, h=1e-3) - g)
    e4 = np.abs(AD.central_difference(*args, h=1e-4) - g)
    assert np.all(e3 / e4 > 50.0), (e3, e4)


def test_no_taper_has_zero_width_gradient():
    args = _case(8, taper_c=0.0)
    _, g = AD.loss_and_grad(*args)
    assert g[2] == 0.0
    G, doms, Xa0, V, y, truth, r, prm = args
    fd = np.zeros(2)
    for i, name in enumerate(("rho", "r_scale")):
        t0 = getattr(prm, name)
        vals = [AD.loss(G, doms, Xa0, V, y, truth, r, L.Params(**{**prm.__dict__, name: t0 * (1 + s * 1e-5)}))
                for s in (1.0, -1.0)]
        fd[i] = (vals[0] - vals[1]) / (2e-5 * t0)
    assert np.allclose(fd, g[:2], rtol=1e-6)


def test_state_adjoint_is_the_transposed_jacobian():
    # <frame_adjoint(Xa_bar), dX> = d/de <Xa_bar, step(Xa + e dX)> at e = 0
    G, doms, Xa0, V, y, truth, r, prm = _case(9, T=1)
    rng = np.random.default_rng(0)
    Xa_bar = rng.standard_normal(Xa0.shape)
    dX = rng.standard_normal(Xa0.shape)
    back, _ = AD.frame_adjoint(G, doms, Xa0, V[0], y[0], r, prm, Xa_bar)
    e = 1e-5
    fp = np.sum(Xa_bar * L.step(G, doms, Xa0 + e * dX, V[0], y[0], r, prm))
    fm = np.sum(Xa_bar * L.step(G, doms, Xa0 - e * dX, V[0], y[0], r, prm))
    assert np.sum(back * dX) == pytest.approx((fp - fm) / (2 * e), rel=1e-7)


def test_inverse_sqrt_adjoint_with_degenerate_cluster():
    # the divided difference -1/(s_i s_j (s_i + s_j)) of l^{-1/2}, applied
    # through the eigenvectors, against a finite difference of A^{-1/2}
    rng = np.random.default_rng(2)
    m = 9
    Y = rng.standard_normal((4, m))
    Y -= Y.mean(axis=1, keepdims=True)
    A = 3.0 * np.eye(m) + Y.T @ Y          # eigenvalue 3 with multiplicity 5
    lam, Q = np.linalg.eigh(A)
    assert np.sum(np.abs(lam - 3.0) < 1e-9) == 5
    Wb = rng.standard_normal((m, m))
    s = np.sqrt(lam)
    F = -1.0 / (np.outer(s, s) * (s[:, None] + s[None, :]))
    Ab = Q @ (F * (Q.T @ (0.5 * (Wb + Wb.T)) @ Q)) @ Q.T
    E = rng.standard_normal((m, m))
    E = E + E.T

    def f(M):
        lm, Qm = np.linalg.eigh(M)
        return (Qm / np.sqrt(lm)) @ Qm.T

    e = 1e-6
    fd = (np.sum(Wb * f(A + e * E)) - np.sum(Wb * f(A - e * E))) / (2 * e)
    assert np.sum(Ab * E) == pytest.approx(fd, rel=1e-7)


def test_loss_adjoint_of_residual_variance():
    rng = np.random.default_rng(4)
    n, m = 30, 6
    X = rng.standard_normal((n, m))
    t = rng.standard_normal(n)
    B = AD.loss_adjoint(X.mean(axis=1), t, 0.3, m)
    dX = rng.standard_normal((n, m))
    e = 1e-6
    fd = 0.3 * (L.residual_variance((X + e * dX).mean(axis=1), t)
                - L.residual_variance((X - e * dX).mean(axis=1), t)) / (2 * e)
    assert np.sum(B * dX) == pytest.approx(fd, rel=1e-8)
