"""The blend-mode gather (a variant of the Sec. 4.2 concatenation) on the GPU
against the oracle: frames through every launch path and transform in both
precisions, the full-size frame with bank noise, an instance of each gather
in one launch, and the refusals.  Bars as for the frame: FP64 1e-10, FP32
1e-4 max relative error."""
import numpy as np
import pytest

from _cases import Case, rel_err
from oracle import blend as BL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def B():
    from paper_1408_7069_amd import binding
    return binding


def _t(a, dt):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dt)).ravel()).to(DEV)


def _ens(f, m):
    return f.get_ensemble().cpu().numpy().astype(np.float64).reshape(-1, m)


@pytest.mark.parametrize("path", ["graph", "direct", "plain", "split"])
@pytest.mark.parametrize("fp64,tol", [(True, 1e-10), (False, 1e-4)])
@pytest.mark.parametrize("geom", [(12, 0.28, 4, 1, 32), (8, None, 2, 0, 20)])
def test_blend_frames(path, fp64, tol, geom):
    N, eps, b, h, m = geom
    case = Case(N, eps, b, h, m, seed=71, fp64=fp64, taper_c=1.5)
    bb = B()
    f = bb.Letkf([case.spec(bb, gather_mode=bb.GATHER_BLEND)])
    f.set_schedule(path == "graph", True)
    X0 = (case.rng.standard_normal((case.G.n_nodes, m)) * 0.5 + case.truth()[:, None]).astype(case.dt)
    f.set_ensemble(_t(X0, case.dt))
    prev = np.asarray(X0, np.float64)
    for k in range(3):
        V, y = case.noise(), case.slopes(case.truth())
        if path == "plain":
            f.step_plain(_t(y, case.dt), V=_t(V, case.dt))
        elif path == "split":
            f.forecast(_t(V, case.dt))
            f.analyse(_t(y, case.dt))
        else:
            f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, m)
        ref = BL.step(case.G, case.doms, prev, np.asarray(V, np.float64), np.asarray(y, np.float64), case.r,
                      case.prm)
        assert rel_err(got.mean(1), ref.mean(1)) <= tol, k
        assert rel_err(got, ref) <= tol, k
        prev = got


@pytest.mark.parametrize("transform", ["NS32", "EVD"])
def test_blend_frame_with_the_other_transforms(transform):
    bb = B()
    case = Case(12, 0.28, 4, 1, 32, seed=73, taper_c=1.5)
    f = bb.Letkf([case.spec(bb, gather_mode=bb.GATHER_BLEND, transform=getattr(bb, "TRANSFORM_" + transform))])
    X0 = (case.rng.standard_normal((case.G.n_nodes, 32)) * 0.5).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    V, y = case.noise(), case.slopes(case.truth())
    f.step(_t(y, np.float32), V=_t(V, np.float32))
    torch.cuda.synchronize()
    ref = BL.step(case.G, case.doms, np.asarray(X0, np.float64), np.asarray(V, np.float64),
                  np.asarray(y, np.float64), case.r, case.prm)
    assert rel_err(_ens(f, 32), ref) <= 1e-4


def test_full_size_blend_frame():
    # 80x80, 28 % obscuration, m = 64, bank noise, graph replay
    case = Case(80, 0.28, 4, 1, 64, seed=75)
    bb = B()
    f = bb.Letkf([case.spec(bb, gather_mode=bb.GATHER_BLEND)])
    n = case.G.n_nodes
    X0 = (case.rng.standard_normal((n, 64)) * 0.3).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    f.set_frame(4)
    y = case.slopes(case.truth())
    f.step(_t(y, np.float32))
    torch.cuda.synchronize()
    assert f.get_frame() == 5
    ref = BL.step(case.G, case.doms, np.asarray(X0, np.float64), case.bank_V(4), np.asarray(y, np.float64),
                  case.r, case.prm)
    got = _ens(f, 64)
    assert rel_err(got.mean(1), ref.mean(1)) <= 1e-4
    assert rel_err(got, ref) <= 1e-4


def test_both_gathers_in_one_launch():
    # a concatenating instance with the piston step and a blending one
    from oracle import letkf as ol
    bb = B()
    c0 = Case(12, 0.28, 4, 1, 32, seed=77, piston=True)
    c1 = Case(10, None, 2, 1, 24, seed=78)
    f = bb.Letkf([c0.spec(bb), c1.spec(bb, gather_mode=bb.GATHER_BLEND)])
    n0 = c0.G.n_nodes
    prev = f.get_ensemble().cpu().numpy().astype(np.float64)
    for k in range(2):
        V = [c0.noise(), c1.noise()]
        ys = [c0.slopes(c0.truth()), c1.slopes(c1.truth())]
        frame = f.get_frame()
        f.step(_t(np.concatenate([y.ravel() for y in ys]), np.float32),
               V=_t(np.concatenate([v.ravel() for v in V]), np.float32))
        torch.cuda.synchronize()
        assert f.get_frame() == frame + 1      # advanced once per frame
        got = f.get_ensemble().cpu().numpy().astype(np.float64)
        r0 = ol.step(c0.G, c0.doms, prev[:n0 * 32].reshape(-1, 32), np.asarray(V[0], np.float64),
                     np.asarray(ys[0], np.float64), c0.r, c0.prm)
        r1 = BL.step(c1.G, c1.doms, prev[n0 * 32:].reshape(-1, 24), np.asarray(V[1], np.float64),
                     np.asarray(ys[1], np.float64), c1.r, c1.prm)
        assert rel_err(got[:n0 * 32].reshape(-1, 32), r0) <= 1e-4, k
        assert rel_err(got[n0 * 32:].reshape(-1, 24), r1) <= 1e-4, k
        prev = got


def test_blend_refusals():
    bb = B()
    case = Case(8, None, 2, 1, 20, seed=79)
    for kw in ({"gather_mode": 2}, {"gather_mode": 1, "piston": True}):
        with pytest.raises(Exception):
            bb.Letkf([case.spec(bb, **kw)])
    h = bb.Letkf([case.spec(bb, gather_mode=bb.GATHER_BLEND)])
    xa = torch.zeros(h.sizes["ensemble_elems"], dtype=torch.float32, device=DEV)
    y = _t(case.slopes(case.truth()), np.float32)
    th = torch.zeros(3, dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        h.adjoint(xa, y, torch.zeros_like(xa), th, 0)
