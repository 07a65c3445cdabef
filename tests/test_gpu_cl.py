"""Covariance localisation (Sec. 4: the prior covariance tapered by a Schur
product) on the GPU against the oracle: frames through every launch path in
both precisions, with and without the taper and the piston step, the
full-size frame with bank noise, and the refusals.  Bars as for the frame:
FP64 1e-10, FP32 1e-4 max relative error."""
import numpy as np
import pytest

from _cases import Case, rel_err
from oracle import cl as CL

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
@pytest.mark.parametrize("geom", [(12, 0.28, 4, 1, 32, 3.0, True), (8, None, 2, 1, 20, 0.0, False)])
def test_cl_frames(path, fp64, tol, geom):
    N, eps, b, h, m, c, piston = geom
    case = Case(N, eps, b, h, m, seed=81, fp64=fp64, taper_c=c, piston=piston)
    bb = B()
    f = bb.Letkf([case.spec(bb, localisation=bb.LOCALISATION_COVARIANCE)])
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
        ref = CL.step(case.G, case.doms, prev, np.asarray(V, np.float64), np.asarray(y, np.float64), case.r,
                      case.prm)
        assert rel_err(got.mean(1), ref.mean(1)) <= tol, k
        assert rel_err(got, ref) <= tol, k
        assert f.status()[0] == bb.OK
        prev = got


@pytest.mark.parametrize("path", ["graph", "plain"])
@pytest.mark.parametrize("fp64,tol", [(True, 1e-10), (False, 1e-4)])
def test_cl_frames_large_domains(path, fp64, tol):
    """5 x 5 domains on a square 15 x 15 grid: up to 36 owned nodes, so 37
    right-hand sides in the solves (a chunk of eight a wave and a second one),
    and up to 49 observation subapertures, p = 98 slopes (past row 64; seven
    Cholesky panels, the last a short one)."""
    case = Case(15, None, 5, 1, 48, seed=83, fp64=fp64, taper_c=3.0, piston=True)
    assert max(len(d.owned) for d in case.doms) + 1 > 32
    assert 2 * max(len(d.obs_subaps) for d in case.doms) > 64
    bb = B()
    f = bb.Letkf([case.spec(bb, localisation=bb.LOCALISATION_COVARIANCE)])
    f.set_schedule(path == "graph", True)
    X0 = (case.rng.standard_normal((case.G.n_nodes, case.m)) * 0.5 + case.truth()[:, None]).astype(case.dt)
    f.set_ensemble(_t(X0, case.dt))
    prev = np.asarray(X0, np.float64)
    for k in range(2):
        V, y = case.noise(), case.slopes(case.truth())
        if path == "plain":
            f.step_plain(_t(y, case.dt), V=_t(V, case.dt))
        else:
            f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        ref = CL.step(case.G, case.doms, prev, np.asarray(V, np.float64), np.asarray(y, np.float64), case.r,
                      case.prm)
        assert rel_err(got.mean(1), ref.mean(1)) <= tol, k
        assert rel_err(got, ref) <= tol, k
        assert f.status()[0] == bb.OK
        prev = got


def test_cl_launch_forms_agree_bitwise():
    """The covariance-localisation kernel gives the same bits from the graph,
    direct launches (either item order) and one launch per domain: every
    reduction in it has a fixed order."""
    case = Case(15, None, 5, 1, 48, seed=84, taper_c=3.0, piston=True)
    bb = B()
    outs = []
    for mode in ["plain", (True, True), (True, False), (False, True), (False, False)]:
        f = bb.Letkf([case.spec(bb, localisation=bb.LOCALISATION_COVARIANCE)])
        rng = np.random.default_rng(1)
        for _k in range(2):
            y = (rng.standard_normal(case.G.n_slopes) * 2).astype(np.float32)
            if mode == "plain":
                f.step_plain(_t(y, np.float32), V=None)
            else:
                f.set_schedule(*mode)
                f.step(_t(y, np.float32), V=None)
        torch.cuda.synchronize()
        outs.append(f.get_ensemble().cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


def test_full_size_cl_frame():
    # 80x80, 28 % obscuration, m = 64, 2-pitch taper, bank noise, graph
    # replay, pistons
    case = Case(80, 0.28, 4, 1, 64, seed=83, taper_c=2.0, piston=True)
    bb = B()
    f = bb.Letkf([case.spec(bb, localisation=bb.LOCALISATION_COVARIANCE)])
    n = case.G.n_nodes
    X0 = (case.rng.standard_normal((n, 64)) * 0.3).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    f.set_frame(6)
    y = case.slopes(case.truth())
    f.step(_t(y, np.float32))
    torch.cuda.synchronize()
    ref = CL.step(case.G, case.doms, np.asarray(X0, np.float64), case.bank_V(6), np.asarray(y, np.float64),
                  case.r, case.prm)
    got = _ens(f, 64)
    assert rel_err(got.mean(1), ref.mean(1)) <= 1e-4
    assert rel_err(got, ref) <= 1e-4


def test_cl_refusals():
    bb = B()
    case = Case(8, None, 2, 1, 20, seed=85)
    for kw in ({"localisation": 4}, {"localisation": 1, "gather_mode": 1},
               {"localisation": 1, "model": 1}):
        with pytest.raises(Exception):
            bb.Letkf([case.spec(bb, **kw)])
    with pytest.raises(Exception):
        bb.Letkf([case.spec(bb, localisation=1), case.spec(bb)])   # mixed localisations
    h = bb.Letkf([case.spec(bb, localisation=bb.LOCALISATION_COVARIANCE)])
    xa = torch.zeros(h.sizes["ensemble_elems"], dtype=torch.float32, device=DEV)
    y = _t(case.slopes(case.truth()), np.float32)
    th = torch.zeros(3, dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        h.adjoint(xa, y, torch.zeros_like(xa), th, 0)
