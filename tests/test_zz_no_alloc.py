"""letkf_adjoint_noalloc, the adjoint for callers that cannot allocate, against
letkf_adjoint through the C ABI: two calls in a row on one device (an 80x80
FP32 handle, then a smaller 12x12 FP64 one, so the second runs on scratch the
first left behind), each equal bit for bit to letkf_adjoint on the same
inputs (the same kernels in the same order; only the scratch differs); and
the refusal of a handle whose buffers exceed the fixed scratch."""
import numpy as np
import pytest

from _cases import Case

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def B():
    from paper_1408_7069_amd import binding
    return binding


def _t(a, dt):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dt)).ravel()).to(DEV)


def _inputs(case, seed):
    rng = np.random.default_rng(seed)
    n, m = case.G.n_nodes, case.m
    xa_prev = (rng.standard_normal((n, m)) * 0.5 + case.truth()[:, None]).astype(case.dt)
    V = case.noise()
    y = case.slopes(case.truth())
    xbar = rng.standard_normal((n, m)).astype(case.dt)
    return xa_prev, V, y, xbar


@pytest.mark.parametrize("noalloc_first", [True, False])
def test_noalloc_adjoint_equals_letkf_adjoint_twice_in_a_row(noalloc_first):
    bb = B()
    cases = [Case(80, 0.28, 4, 1, 64, seed=71, fp64=False, taper_c=2.0, piston=True),
             Case(12, 0.28, 4, 1, 32, seed=72, fp64=True, taper_c=1.5, piston=True)]
    for i, case in enumerate(cases):
        print(f"noalloc adjoint: case {i} N={case.N} m={case.m} fp64={case.fp64}", flush=True)
        f = bb.Letkf([case.spec(bb)])
        xa_prev, V, y, xbar = _inputs(case, 100 + i)
        outs = {}
        order = ["noalloc", "alloc"] if noalloc_first else ["alloc", "noalloc"]
        for kind in order:
            xb = _t(xbar, case.dt)
            th = torch.zeros(3, dtype=torch.float64, device=DEV)
            call = f.adjoint_noalloc if kind == "noalloc" else f.adjoint
            call(_t(xa_prev, case.dt), _t(y, case.dt), xb, th, frame=3, V=_t(V, case.dt))
            torch.cuda.synchronize()
            outs[kind] = (xb.cpu().numpy(), th.cpu().numpy())
        assert np.all(np.isfinite(outs["alloc"][0])) and np.any(outs["alloc"][0] != 0)
        assert np.array_equal(outs["noalloc"][0], outs["alloc"][0]), i
        assert np.array_equal(outs["noalloc"][1], outs["alloc"][1]), i
        f.close()


def test_noalloc_adjoint_refuses_a_handle_beyond_its_scratch():
    bb = B()
    case = Case(80, 0.28, 4, 1, 64, seed=73, fp64=True)
    f = bb.Letkf([case.spec(bb)] * 2)          # two 80x80 FP64 instances: 26.5 MB
    n = f.sizes["ensemble_elems"]
    z = torch.zeros(n, dtype=torch.float64, device=DEV)
    y = torch.zeros(f.sizes["n_slopes"], dtype=torch.float64, device=DEV)
    th = torch.zeros(6, dtype=torch.float64, device=DEV)
    with pytest.raises(bb.LetkfError) as e:
        f.adjoint_noalloc(z, y, z.clone(), th, frame=0, V=z)
    assert e.value.code == bb.E_INVAL
    assert "scratch" in bb.lib.letkf_last_error().decode()
    f.close()
