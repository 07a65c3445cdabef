"""Variants that meet in one frame, on the GPU against the oracle composed
from the same parts: the blend-mode gather with the closed loop and with the
AR(2) model, covariance localisation with the AR(2) model and with the
online refit.  Bars as for the frame: FP64 1e-10, FP32 1e-4."""
import numpy as np
import pytest

from _cases import Case, rel_err
from oracle import ar2
from oracle import blend as BL
from oracle import cl as CL
from oracle import delayed as DL
from oracle import letkf as ol
from oracle import piston
from oracle import refit as RF

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = [(True, 1e-10), (False, 1e-4)]


def B():
    from paper_1408_7069_amd import binding
    return binding


def _t(a, dt):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dt)).ravel()).to(DEV)


def _ens(f, m):
    return f.get_ensemble().cpu().numpy().astype(np.float64).reshape(-1, m)


def _start(case, f):
    X0 = (case.rng.standard_normal((case.G.n_nodes, case.m)) * 0.5 + case.truth()[:, None]).astype(case.dt)
    f.set_ensemble(_t(X0, case.dt))
    return np.asarray(X0, np.float64)


@pytest.mark.parametrize("fp64,tol", PREC)
def test_blend_with_the_closed_loop(fp64, tol):
    case = Case(12, 0.28, 4, 1, 32, seed=91, fp64=fp64, taper_c=1.5)
    bb = B()
    f = bb.Letkf([case.spec(bb, model=bb.MODEL_CLOSED_LOOP, gather_mode=bb.GATHER_BLEND)])
    Xa = _start(case, f)
    n = case.G.n_nodes
    u1, u2 = case.rng.standard_normal(n), case.rng.standard_normal(n)
    f.set_command(_t(u1, case.dt), _t(u2, case.dt))
    u1, u2 = np.asarray(u1, case.dt).astype(np.float64), np.asarray(u2, case.dt).astype(np.float64)
    for k in range(3):
        V, y = case.noise(), case.slopes(case.truth())
        f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        Xb = ol.forecast(Xa, np.asarray(V, np.float64), case.prm.a)
        ref = BL.analysis(case.G, case.doms, Xb, np.asarray(y, np.float64), case.r, case.prm, u_prev2=u2)
        assert rel_err(got, ref) <= tol, k
        cmd = f.get_command().cpu().numpy().astype(np.float64)
        assert rel_err(cmd, DL.command(ref, case.prm.a)) <= tol, k
        u2, u1, Xa = u1, cmd, got


@pytest.mark.parametrize("fp64,tol", PREC)
def test_blend_with_ar2(fp64, tol):
    a1, a2 = ar2.yule_walker(0.98, 0.95)
    case = Case(12, 0.28, 4, 1, 32, seed=92, fp64=fp64, taper_c=1.5)
    case.prm.a = a1
    bb = B()
    f = bb.Letkf([case.spec(bb, ar_coeff=a1, ar2_coeff=a2, gather_mode=bb.GATHER_BLEND)])
    Xa = Xp = _start(case, f)
    for k in range(3):
        V, y = case.noise(), case.slopes(case.truth())
        f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        Xb = ar2.forecast(Xa, Xp, np.asarray(V, np.float64), a1, a2)
        ref = BL.analysis(case.G, case.doms, Xb, np.asarray(y, np.float64), case.r, case.prm)
        assert rel_err(got, ref) <= tol, k
        Xp, Xa = Xa, got


@pytest.mark.parametrize("fp64,tol", PREC)
def test_covariance_localisation_with_ar2(fp64, tol):
    a1, a2 = ar2.yule_walker(0.98, 0.95)
    case = Case(12, 0.28, 4, 1, 32, seed=93, fp64=fp64, taper_c=3.0, piston=True)
    case.prm.a = a1
    bb = B()
    f = bb.Letkf([case.spec(bb, ar_coeff=a1, ar2_coeff=a2, localisation=bb.LOCALISATION_COVARIANCE)])
    Xa = Xp = _start(case, f)
    for k in range(3):
        V, y = case.noise(), case.slopes(case.truth())
        f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        Xb = ar2.forecast(Xa, Xp, np.asarray(V, np.float64), a1, a2)
        ref = CL.analysis(case.G, case.doms, Xb, np.asarray(y, np.float64), case.r, case.prm)
        ref = piston.remove(case.G, case.doms, ref, np.asarray(y, np.float64))
        assert rel_err(got, ref) <= tol, k
        Xp, Xa = Xa, got


@pytest.mark.parametrize("fp64,tol", PREC)
def test_covariance_localisation_with_the_refit(fp64, tol):
    a0 = 0.95
    case = Case(12, 0.28, 4, 1, 32, seed=94, fp64=fp64, taper_c=3.0, piston=True, a=a0)
    bb = B()
    f = bb.Letkf([case.spec(bb, refit_forgetting=0.9, localisation=bb.LOCALISATION_COVARIANCE)])
    Xa = _start(case, f)
    rg = RF.ArRefit(a0, 0.9)
    for k in range(3):
        V, y = case.noise(), case.slopes(case.truth())
        f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        Xb = ol.forecast(Xa, rg.noise_scale() * np.asarray(V, np.float64), rg.a)
        ref = CL.analysis(case.G, case.doms, Xb, np.asarray(y, np.float64), case.r, case.prm)
        ref = piston.remove(case.G, case.doms, ref, np.asarray(y, np.float64))
        assert rel_err(got, ref) <= tol, k
        rg.update(got.mean(axis=1), Xa.mean(axis=1))
        assert abs(f.get_model()[0][0] - rg.a) <= 1e-9 * rg.a, k
        Xa = got
