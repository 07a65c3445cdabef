"""The AR(2) forecast on the GPU against the oracle: frames through every
launch path in both precisions, the full-size frame, and the refusals.
Bars as for the frame: FP64 1e-10, FP32 1e-4."""
import numpy as np
import pytest

from _cases import Case, rel_err
from oracle import ar2

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
def test_ar2_frames(path, fp64, tol):
    a1, a2 = ar2.yule_walker(0.98, 0.95)
    # (the case's noise keeps its AR(1) scaling; only the instance and the
    # oracle take the AR(2) coefficients)
    case = Case(12, 0.28, 4, 1, 32, seed=51, fp64=fp64, piston=True, taper_c=1.5)
    case.prm.a = a1
    bb = B()
    f = bb.Letkf([case.spec(bb, ar_coeff=a1, ar2_coeff=a2)])
    f.set_schedule(path == "graph", True)
    X0 = (case.rng.standard_normal((case.G.n_nodes, case.m)) * 2).astype(case.dt)
    f.set_ensemble(_t(X0, case.dt))          # sets the history too
    Xa = Xp = np.asarray(X0, np.float64)
    for k in range(4):
        V, y = case.noise(), case.slopes(case.truth())
        if path == "plain":
            f.step_plain(_t(y, case.dt), V=_t(V, case.dt))
        elif path == "split":
            f.forecast(_t(V, case.dt))
            f.analyse(_t(y, case.dt))
        else:
            f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, case.m)
        ref = ar2.step(case.G, case.doms, Xa, Xp, np.asarray(V, np.float64), np.asarray(y, np.float64),
                       case.r, case.prm, a2)
        assert rel_err(got.mean(1), ref.mean(1)) <= tol, k
        assert rel_err(got, ref) <= tol, k
        Xp, Xa = Xa, got                     # the GPU's own history on both sides


def test_full_size_ar2_frame():
    a1, a2 = ar2.yule_walker(0.995, 0.985)
    case = Case(80, 0.28, 4, 1, 64, seed=53, piston=True)
    case.prm.a = a1
    bb = B()
    f = bb.Letkf([case.spec(bb, ar_coeff=a1, ar2_coeff=a2)])
    X0 = (case.rng.standard_normal((case.G.n_nodes, 64)) * 0.3).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    f.set_frame(2)
    y = case.slopes(case.truth())
    f.step(_t(y, np.float32))
    torch.cuda.synchronize()
    Xa = np.asarray(X0, np.float64)
    ref = ar2.step(case.G, case.doms, Xa, Xa, case.bank_V(2), np.asarray(y, np.float64), case.r, case.prm, a2)
    got = _ens(f, 64)
    assert rel_err(got.mean(1), ref.mean(1)) <= 1e-4
    assert rel_err(got, ref) <= 1e-4


def test_ar2_refusals():
    bb = B()
    case = Case(8, None, 2, 1, 20, seed=55)
    with pytest.raises(Exception):
        bb.Letkf([case.spec(bb, ar2_coeff=1.0)])
    with pytest.raises(Exception):
        bb.Letkf([case.spec(bb, ar2_coeff=0.3, model=bb.MODEL_CLOSED_LOOP)])
    g = bb.Letkf([case.spec(bb, ar2_coeff=0.3)])
    xa = torch.zeros(g.sizes["ensemble_elems"], dtype=torch.float32, device=DEV)
    y = _t(case.slopes(case.truth()), np.float32)
    with pytest.raises(Exception):
        g.adjoint(xa, y, torch.zeros_like(xa), torch.zeros(3, dtype=torch.float64, device=DEV), 0)
