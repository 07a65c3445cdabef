"""Pins of the AR(2) turbulence model (Sec. 6 names it as the extension of
the AR(1) model of Sec. 2.2): the AR(1) limit, the Yule-Walker relations and
the innovation scale of a stationary unit-variance process, and the
stationarity of the synthetic AR(2) truth."""
import numpy as np
import pytest

from oracle import ar2
from oracle import geometry as geo
from oracle import letkf as ol
from paper_1408_7069_amd import workload as wl


def test_a2_zero_is_the_ar1_frame():
    G = geo.geometry_for(12, 0.28)
    doms = geo.domains(G, 4, 1)
    rng = np.random.default_rng(1)
    prm = ol.Params(a=0.97, rho=1.05, b=4, h=1, piston=True, taper_c=1.5)
    Xa, Xp = rng.standard_normal((2, G.n_nodes, 24))
    V = 0.3 * rng.standard_normal((G.n_nodes, 24))
    r = np.full(G.n_slopes, 0.02)
    y = rng.standard_normal(G.n_slopes)
    assert np.allclose(ar2.step(G, doms, Xa, Xp, V, y, r, prm, 0.0), ol.step(G, doms, Xa, V, y, r, prm),
                       atol=1e-13)


@pytest.mark.parametrize("rho1,rho2", [(0.95, 0.85), (0.99, 0.97), (0.6, 0.1)])
def test_yule_walker_and_the_innovation_scale(rho1, rho2):
    a1, a2 = ar2.yule_walker(rho1, rho2)
    assert a1 / (1 - a2) == pytest.approx(rho1) and a1 * rho1 + a2 == pytest.approx(rho2)
    s = ar2.innovation_std(a1, a2)
    # a long scalar realisation: unit variance and the two correlations
    rng = np.random.default_rng(3)
    n = 400_000
    e = rng.standard_normal(n) * s
    x = np.empty(n)
    x[0] = rng.standard_normal()
    x[1] = rho1 * x[0] + np.sqrt(1 - rho1 * rho1) * rng.standard_normal()
    for k in range(2, n):
        x[k] = a1 * x[k - 1] + a2 * x[k - 2] + e[k]
    x = x[2000:]
    assert np.var(x) == pytest.approx(1.0, abs=0.05)
    assert np.corrcoef(x[1:], x[:-1])[0, 1] == pytest.approx(rho1, abs=0.01)
    assert np.corrcoef(x[2:], x[:-2])[0, 1] == pytest.approx(rho2, abs=0.015)


def test_ar2_truth_is_stationary_von_karman():
    # 400 independent short runs of a 4x4-subaperture grid: every frame has the
    # von Karman variance of the generator, consecutive frames rho1
    a1, a2 = ar2.yule_walker(0.9, 0.75)
    C0 = wl.vk_covariance(10, 0.4, 0.15, 25.0)[0, 0]
    rng = np.random.default_rng(4)
    runs = np.array([wl.ar2_truth(4, 6, 0.4, 0.15, 25.0, a1, a2, rng) for _ in range(400)])
    v = runs[:, :, 2, 2]
    for k in range(6):
        assert np.var(v[:, k]) == pytest.approx(C0, rel=0.15), k
    c = np.mean([np.corrcoef(v[:, k], v[:, k + 1])[0, 1] for k in range(5)])
    assert c == pytest.approx(0.9, abs=0.03)
