"""Pins of the oracle's geometry (G1-G6) against numbers printed in the paper
and closed-form properties of the Fried slope operator."""
import json
import os

import numpy as np
import pytest

from oracle import geometry as geo

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_pupil_16m_counts():
    g = GOLD["geometry_16m"]
    G = geo.Geometry(geo.pupil_mask(g["n_sub"], g["obscuration"]))
    assert G.n_subaps == g["valid_subapertures"]
    assert G.n_slopes == g["slopes"]
    assert G.n_nodes == g["valid_actuators"]
    assert 2 * G.n_nodes == g["state_dim_two_copies"]


def test_pupil_40m_counts():
    g = GOLD["geometry_40m"]
    G = geo.Geometry(geo.pupil_mask(g["n_sub"], g["obscuration"]))
    assert G.n_slopes == g["slopes"]
    assert 2 * G.n_nodes == g["state_dim_two_copies"]


@pytest.mark.parametrize("ss", [32, 128])
def test_mask_stable_in_sampling(ss):
    # no subaperture sits near the 50 % threshold for these pupils
    for N, eps in [(32, 0.0), (80, 0.28)]:
        assert np.array_equal(geo.pupil_mask(N, eps, ss=ss), geo.pupil_mask(N, eps))


def test_partition_counts_of_actuator_grid():
    # a P x P partition of the (N+1)^2 actuator grid has the printed number of
    # non-empty domains: pins the shape of the valid-node mask at the edge
    for case in GOLD["partition_counts"]["cases"]:
        N, P = case["n_sub"], case["P"]
        G = geo.Geometry(geo.pupil_mask(N, 0.0))
        blocks = {(i * P // (N + 1), j * P // (N + 1)) for i, j in G.node_coords()}
        assert len(blocks) == case["domains"]


def test_small_workload_geometries():
    # square 8x8 with 2x2 domains, halo 1: 64 subaps, 128 slopes, 81 nodes, 16 domains
    G = geo.Geometry(geo.square_mask(8))
    assert (G.n_subaps, G.n_slopes, G.n_nodes) == (64, 128, 81)
    doms = geo.domains(G, 2, 1)
    assert len(doms) == 16
    assert sorted({len(d.owned) for d in doms}) == [4, 6, 9]
    assert min(len(d.obs) for d in doms) == 18 and max(len(d.obs) for d in doms) == 32
    # 80x80 with 28 % obscuration, 4x4 domains, halo 1 (rule-derived counts)
    G = geo.Geometry(geo.pupil_mask(80, 0.28))
    assert (G.n_subaps, G.n_nodes) == (4632, 4836)
    doms = geo.domains(G, 4, 1)
    assert len(doms) == 332
    assert max(len(d.obs) for d in doms) == 72
    assert sum(len(d.obs) for d in doms) == 20644


def test_domains_partition_the_nodes():
    G = geo.Geometry(geo.pupil_mask(24, 0.3))
    doms = geo.domains(G, 4, 1)
    owned = np.concatenate([d.owned for d in doms])
    assert np.array_equal(np.sort(owned), np.arange(G.n_nodes))
    # every slope touching an owned node is in that domain's observation region
    D = geo.slope_matrix(G)
    for d in doms:
        touching = np.nonzero(np.abs(D[:, d.owned]).sum(axis=1))[0]
        assert set(touching) <= set(d.obs.tolist())


def test_fried_operator_closed_forms():
    G = geo.Geometry(geo.pupil_mask(16, 0.2))
    ij = G.node_coords()
    D = geo.slope_matrix(G)
    ps = G.n_subaps
    # piston is unseen
    assert np.abs(D @ np.ones(G.n_nodes)).max() == 0.0
    # tilt along columns (x) and rows (y)
    sx = D @ ij[:, 1].astype(float)
    assert np.allclose(sx[:ps], 1.0) and np.allclose(sx[ps:], 0.0)
    sy = D @ ij[:, 0].astype(float)
    assert np.allclose(sy[:ps], 0.0) and np.allclose(sy[ps:], 1.0)
    # waffle is in the null space of the Fried geometry
    waffle = (-1.0) ** (ij[:, 0] + ij[:, 1])
    assert np.abs(D @ waffle).max() == 0.0
    # four non-zeros of magnitude 1/2 per row
    assert np.all((np.abs(D) > 0).sum(axis=1) == 4) and np.all(np.abs(D[D != 0]) == 0.5)
    # the stencil routine equals the matrix
    x = np.random.default_rng(0).standard_normal((G.n_nodes, 3))
    assert np.allclose(geo.apply_slopes(G, x), D @ x, atol=1e-14)


def test_fried_rank_deficiency():
    # square N x N Fried geometry: null space = piston + waffle, so rank n - 2
    G = geo.Geometry(geo.square_mask(6))
    D = geo.slope_matrix(G)
    assert np.linalg.matrix_rank(D) == G.n_nodes - 2


def test_gaspari_cohn_properties():
    z = np.linspace(0, 2.5, 2501)
    f = geo.gaspari_cohn(z)
    assert f[0] == 1.0 and np.all(f[z >= 2.0] == 0.0)
    assert np.all(np.diff(f) <= 1e-15)
    # value, first and second derivative continuous at z = 1 and z = 2
    for z0 in (1.0, 2.0):
        e = 1e-6
        lo, hi = geo.gaspari_cohn(np.array([z0 - e])), geo.gaspari_cohn(np.array([z0 + e]))
        assert abs(lo[0] - hi[0]) < 1e-5
        dl, dh = geo.gaspari_cohn_deriv(np.array([z0 - e])), geo.gaspari_cohn_deriv(np.array([z0 + e]))
        assert abs(dl[0] - dh[0]) < 1e-5
    # the analytic derivative matches finite differences
    zz = np.array([0.3, 0.9, 1.2, 1.7, 1.95])
    fd = (geo.gaspari_cohn(zz + 1e-6) - geo.gaspari_cohn(zz - 1e-6)) / 2e-6
    assert np.allclose(fd, geo.gaspari_cohn_deriv(zz), atol=1e-8)
    # a correlation function: positive semi-definite on scattered points
    pts = np.random.default_rng(1).uniform(0, 6, (120, 2))
    dist = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1))
    C = geo.gaspari_cohn(dist / 1.5)
    assert np.linalg.eigvalsh(C).min() > -1e-10


def test_taper_off_is_one_and_on_is_local():
    G = geo.Geometry(geo.pupil_mask(20, 0.2))
    doms = geo.domains(G, 4, 2)
    for d in doms:
        assert np.all(geo.taper(d, 4, 0.0) == 1.0)
        f = geo.taper(d, 4, 2.0)
        dist = geo.taper_dist(d, 4)
        assert np.all((f > 0) == (dist < 4.0))


@pytest.mark.parametrize("N,eps", [(6, None), (10, 0.3)])
def test_slope_adjoint_is_the_transpose(N, eps):
    # D^T by scatter against the dense matrix, and <D x, s> = <x, D^T s>
    G = geo.geometry_for(N, eps)
    rng = np.random.default_rng(N)
    D = geo.slope_matrix(G)
    s = rng.standard_normal((G.n_slopes, 3))
    assert np.allclose(geo.apply_slopes_adjoint(G, s), D.T @ s, atol=1e-14)
    x = rng.standard_normal(G.n_nodes)
    s1 = s[:, 0]
    assert np.dot(geo.apply_slopes(G, x), s1) == pytest.approx(np.dot(x, geo.apply_slopes_adjoint(G, s1)),
                                                                rel=1e-13)
