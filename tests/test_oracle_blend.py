"""Pins of the blend-mode gather (a variant of the Sec. 4.2 concatenation):
one domain is the global analysis, the tent weights, planted pistons are
removed exactly, no information keeps the forecast, the alignment's normal
equations, and the blended filter loop against concatenation."""
import numpy as np
import pytest

from oracle import blend as BL
from oracle import geometry as geo
from oracle import letkf as ol
from paper_1408_7069_amd import workload as wl


def _ens(G, m, rng, scale=1.0):
    return rng.standard_normal((G.n_nodes, m)) * scale


def test_one_domain_is_the_global_analysis():
    G = geo.geometry_for(6, None)
    doms = geo.domains(G, 6, 0)
    assert len(doms) == 1
    rng = np.random.default_rng(1)
    Xb = _ens(G, 12, rng) + rng.standard_normal(G.n_nodes)[:, None]
    y = geo.apply_slopes(G, rng.standard_normal(G.n_nodes)) + 0.1 * rng.standard_normal(G.n_slopes)
    r = np.full(G.n_slopes, 0.01)
    prm = ol.Params(b=6, h=0, rho=1.05)
    assert np.abs(BL.analysis(G, doms, Xb, y, r, prm) - ol.analysis(G, doms, Xb, y, r, prm)).max() <= 1e-12


def test_tent_weights():
    G = geo.geometry_for(12, None)
    b, h = 4, 1
    ij = G.node_coords()
    for dom in geo.domains(G, b, h):
        P = BL.patch_nodes(G, dom)
        assert set(dom.owned) <= set(P)
        om = BL.weights(G, dom, b, h, P)
        assert np.all(om > 0) and np.all(om <= 1)
        assert np.all(BL.weights(G, dom, b, h, dom.owned) == 1.0)
        I, J = dom.block
        for k, n in enumerate(P):
            i, j = ij[n]
            di = max(0, I * b - i, i - (I * b + b - 1 if I < 2 else 12))
            dj = max(0, J * b - j, j - (J * b + b - 1 if J < 2 else 12))
            assert om[k] == pytest.approx((1 - di / 3) * (1 - dj / 3))


def test_planted_pistons_are_removed_exactly():
    # patches that agree up to one constant per domain blend to the common
    # field plus one overall constant
    G = geo.geometry_for(12, 0.2)
    doms = geo.domains(G, 4, 1)
    rng = np.random.default_rng(2)
    T = _ens(G, 5, rng)
    parts, oms = [], []
    for dom in doms:
        P = BL.patch_nodes(G, dom)
        parts.append((P, T[P] + rng.uniform(-5, 5)))
        oms.append(rng.uniform(0.1, 1.0, len(P)))
    out = BL.gather(parts, oms, G.n_nodes)
    off = out - T
    assert np.abs(off - off.mean()).max() <= 1e-12


def test_no_information_keeps_the_forecast():
    G = geo.geometry_for(12, 0.2)
    doms = geo.domains(G, 4, 1)
    rng = np.random.default_rng(3)
    Xb = _ens(G, 16, rng) + 3.0 * rng.standard_normal(G.n_nodes)[:, None]
    y = rng.standard_normal(G.n_slopes)
    r = np.full(G.n_slopes, 1e14)
    out = BL.analysis(G, doms, Xb, y, r, ol.Params(b=4, h=1, rho=1.0))
    assert np.abs(out - Xb).max() <= 1e-9


def test_alignment_solves_the_laplacian_normal_equations():
    # pi solves L pi = r with L the graph Laplacian weighted by the number of
    # shared nodes, r_l the summed mean differences, and has zero sum
    G = geo.geometry_for(12, 0.28)
    doms = geo.domains(G, 4, 1)
    rng = np.random.default_rng(4)
    parts = [(BL.patch_nodes(G, d), None) for d in doms]
    parts = [(P, rng.standard_normal((len(P), 3))) for P, _ in parts]
    pi = BL.alignment(parts, len(doms))
    nd = len(doms)
    L = np.zeros((nd, nd))
    rhs = np.zeros(nd)
    where = {}
    for l, (P, X) in enumerate(parts):
        for k, n in enumerate(P):
            where.setdefault(int(n), []).append((l, X[k].mean()))
    for lst in where.values():
        for l, xl in lst:
            for q, xq in lst:
                if q != l:
                    L[l, l] += 1
                    L[l, q] -= 1
                    rhs[l] += xq - xl
    assert np.abs(L @ pi - rhs).max() <= 1e-10
    assert abs(pi.sum()) <= 1e-10


def test_blended_filter_loop_is_stable_and_close_to_the_piston_step():
    # 12x12 square pupil, 4x4 domains, halo 1, m = 32, a = 0.99: the
    # concatenation without the piston step diverges (its border pistons
    # grow); the aligned blend stays within 30 % of concatenation with the
    # piston step
    N, b, h, m, T, a = 12, 4, 1, 32, 120, 0.99
    G = geo.geometry_for(N, None)
    ij = G.node_coords()
    doms = geo.domains(G, b, h)
    rng = np.random.default_rng(5)
    truth = np.array([g[ij[:, 0], ij[:, 1]] for g in wl.ar1_truth(N, T, 0.4, 0.15, 25.0, a, rng)])
    r = np.full(G.n_slopes, 0.04)
    out = {}
    for name in ("concat", "concat+piston", "blend"):
        rng = np.random.default_rng(9)
        prm = ol.Params(a=a, rho=1.05, b=b, h=h, piston=name == "concat+piston")
        Xa = np.zeros((G.n_nodes, m))
        err = []
        for k in range(T):
            V = np.sqrt(1 - a * a) * np.stack(
                [s[ij[:, 0], ij[:, 1]] for s in wl.vk_screens(2 * (N + 1), 0.4, 0.15, 25.0, m, rng)], 1)
            y = geo.apply_slopes(G, truth[k]) + 0.2 * rng.standard_normal(G.n_slopes)
            Xa = BL.step(G, doms, Xa, V, y, r, prm) if name == "blend" else ol.step(G, doms, Xa, V, y, r, prm)
            err.append(ol.residual_variance(Xa.mean(1), truth[k]))
        out[name] = float(np.mean(err[T // 2:]))
    assert out["concat"] > 100 * out["concat+piston"], out
    assert out["blend"] < 1.3 * out["concat+piston"], out
