"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, validates configurations, and its host planner builds exactly the
oracle's integer maps (node numbering, owners, observation lists)."""
import os

import numpy as np
import pytest

from oracle import geometry as geo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "letkf.h")

binding = pytest.importorskip("paper_1408_7069_amd.binding")


def test_every_declared_symbol_is_exported():
    names = binding.header_symbols(HEADER)
    assert len(names) >= 20
    for n in names:
        assert hasattr(binding.lib, n), n


def test_kernel_argument_blocks_match_their_host_mirrors():
    # analysis, adjoint and piston argument blocks: the kernels' sizeof against
    # the host-side mirrors (separate translation units of the library)
    assert binding.lib.letkf_layout_check() == 0


def test_strerror_and_codes():
    assert binding.lib.letkf_strerror(0) == b"ok"
    for code in range(-6, 0):
        assert binding.lib.letkf_strerror(code) != b"unknown error"


@pytest.mark.parametrize("bad", [dict(m=1), dict(m=129), dict(rho=0.0), dict(r_scale=-1.0),
                                 dict(domain_size=0), dict(halo=-1), dict(domain_size=6, halo=3),
                                 dict(domain_size=11, halo=0),
                                 dict(r_sigma2=0.0), dict(obscuration=1.0), dict(taper_c=-1.0)])
def test_invalid_configs_are_rejected(bad):
    spec = binding.InstanceSpec(n_sub=8, m=16, domain_size=2, halo=1)
    for k, v in bad.items():
        setattr(spec, k, v)
    with pytest.raises(binding.LetkfError) as e:
        binding.plan(spec)
    assert e.value.code == binding.E_INVAL


def test_bank_shape_is_validated():
    spec = binding.InstanceSpec(n_sub=8, m=16, domain_size=2, halo=1,
                                noise_bank=np.zeros((2, 12, 12), np.float32))
    with pytest.raises(binding.LetkfError):
        binding.plan(spec)


CASES = [(8, None, 2, 1), (12, 0.28, 4, 1), (40, 0.14, 4, 1), (80, 0.28, 4, 1), (13, 0.3, 3, 2),
         (17, 0.0, 5, 1), (5, None, 1, 0), (1, None, 1, 0), (33, 0.1, 4, 0),
         # the wide shapes: the paper's 4 x 4 domains with a halo of 2, and
         # domain size plus twice the halo at its limit of 10
         (80, 0.28, 4, 2), (24, 0.28, 6, 2), (30, None, 10, 0), (21, 0.2, 2, 4)]


@pytest.mark.parametrize("N,eps,b,h", CASES)
def test_planner_matches_oracle_bit_exactly(N, eps, b, h):
    G = geo.geometry_for(N, eps)
    doms = geo.domains(G, b, h)
    spec = binding.InstanceSpec(n_sub=N, m=8, domain_size=b, halo=h,
                                obscuration=0.0 if eps is None else eps,
                                mask=geo.square_mask(N) if eps is None else None)
    sizes, maps = binding.plan(spec)
    assert sizes["n_nodes"] == G.n_nodes and sizes["n_slopes"] == G.n_slopes
    assert sizes["n_domains"] == len(doms)
    assert np.array_equal(maps["node_ij"], G.node_coords())
    assert np.array_equal(maps["owner"], geo.owner_map(G, doms))
    obs = [maps["obs_idx"][maps["obs_off"][k]:maps["obs_off"][k + 1]] for k in range(len(doms))]
    own = [maps["own_idx"][maps["own_off"][k]:maps["own_off"][k + 1]] for k in range(len(doms))]
    for d, o, w in zip(doms, obs, own):
        assert np.array_equal(o, d.obs)
        assert np.array_equal(w, d.owned)


def test_planner_takes_a_caller_mask():
    rng = np.random.default_rng(0)
    mask = rng.random((10, 10)) > 0.3
    G = geo.Geometry(mask)
    sizes, maps = binding.plan(binding.InstanceSpec(n_sub=10, m=4, domain_size=2, halo=1, mask=mask))
    assert np.array_equal(maps["node_ij"], G.node_coords())
    assert sizes["n_slopes"] == G.n_slopes
