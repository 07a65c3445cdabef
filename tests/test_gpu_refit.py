"""The online AR(1) refit (Sec. 4.2: the model re-identified while the filter
runs) on the GPU against the oracle: the refitted coefficient from the GPU's
own analyses, every frame's ensemble from the refitted model through every
launch path, in both models and precisions, the full-size frame with bank
noise, mixed instances, restarts, and the refusals.

Bars: the coefficient and noise scale, computed from the same ensembles on
both sides, within 1e-9 relative; ensembles as for the frame, FP64 1e-10,
FP32 1e-4."""
import copy

import numpy as np
import pytest

from _cases import Case, rel_err
from oracle import delayed as DL
from oracle import refit as RF

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


def _truth_seq(case, a_true, T):
    x = [case.truth()]
    for _ in range(T):
        x.append(a_true * x[-1] + np.sqrt(1 - a_true * a_true) * case.truth())
    return x


@pytest.mark.parametrize("path", ["graph", "direct", "plain", "split"])
@pytest.mark.parametrize("fp64,tol", [(True, 1e-10), (False, 1e-4)])
@pytest.mark.parametrize("model", [0, 1])
def test_refit_frames(path, fp64, tol, model):
    a0, f_forget = 0.95, 0.9
    case = Case(12, 0.28, 4, 1, 32, seed=61, fp64=fp64, piston=True, a=a0, taper_c=1.5)
    bb = B()
    f = bb.Letkf([case.spec(bb, model=model, refit_forgetting=f_forget)])
    f.set_schedule(path == "graph", True)
    n, m = case.G.n_nodes, case.m
    X0 = (case.rng.standard_normal((n, m)) * 0.5 + case.truth()[:, None]).astype(case.dt)
    f.set_ensemble(_t(X0, case.dt))
    u1 = u2 = np.zeros(n)
    prev = np.asarray(X0, np.float64)
    rg = RF.ArRefit(a0, f_forget)          # fed with the GPU's own analyses
    truth = _truth_seq(case, 0.995, 6)
    for k in range(6):
        V, y = case.noise(), case.slopes(truth[k])
        a_used = rg.a
        if path == "plain":
            f.step_plain(_t(y, case.dt), V=_t(V, case.dt))
        elif path == "split":
            f.forecast(_t(V, case.dt))
            f.analyse(_t(y, case.dt))
        else:
            f.step(_t(y, case.dt), V=_t(V, case.dt))
        torch.cuda.synchronize()
        got = _ens(f, m)
        ref, a_ref = RF.frame(case.G, case.doms, prev, np.asarray(V, np.float64), np.asarray(y, np.float64),
                              case.r, case.prm, copy.deepcopy(rg), u_prev2=u2 if model == 1 else None)
        assert a_ref == a_used
        assert rel_err(got, ref) <= tol, k
        if model == 1:
            cmd = f.get_command().cpu().numpy().astype(np.float64)
            assert rel_err(cmd, DL.command(ref, a_used)) <= tol, k
            u2, u1 = u1, cmd
        rg.update(got.mean(axis=1), prev.mean(axis=1))
        a, vs = f.get_model()
        assert abs(a[0] - rg.a) <= 1e-9 * rg.a, k
        assert abs(vs[0] - rg.noise_scale()) <= 1e-9 * rg.noise_scale(), k
        prev = got
    assert rg.a != a0                      # the model did move


def test_full_size_refit_frames_with_bank_noise():
    # 80x80, 28 % obscuration, m = 64, bank noise, graph replay, pistons: the
    # third frame uses a refitted a and the bank scaled for it
    a0 = 0.99
    case = Case(80, 0.28, 4, 1, 64, seed=63, piston=True, a=a0)
    bb = B()
    f = bb.Letkf([case.spec(bb, refit_forgetting=0.95)])
    n = case.G.n_nodes
    truth = _truth_seq(case, 0.9, 3)
    X0 = (case.rng.standard_normal((n, 64)) * 0.3 + truth[0][:, None]).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    prev = np.asarray(X0, np.float64)
    rg = RF.ArRefit(a0, 0.95)
    for k in range(3):
        y = case.slopes(truth[k + 1])
        frame = f.get_frame()
        f.step(_t(y, np.float32))
        torch.cuda.synchronize()
        got = _ens(f, 64)
        ref, _ = RF.frame(case.G, case.doms, prev, case.bank_V(frame), np.asarray(y, np.float64), case.r,
                          case.prm, copy.deepcopy(rg))
        assert rel_err(got.mean(1), ref.mean(1)) <= 1e-4, k
        assert rel_err(got, ref) <= 1e-4, k
        rg.update(got.mean(axis=1), prev.mean(axis=1))
        a, vs = f.get_model()
        assert abs(a[0] - rg.a) <= 1e-9 * rg.a and abs(vs[0] - rg.noise_scale()) <= 1e-9 * rg.noise_scale()
        prev = got
    assert rg.a < a0 and rg.noise_scale() > 1.0


def test_mixed_instances_reset_and_tuning_keep_the_model():
    bb = B()
    c0 = Case(12, 0.28, 4, 1, 32, seed=65, piston=True, a=0.97)
    c1 = Case(10, None, 2, 1, 24, seed=66, piston=True, a=0.98)
    f = bb.Letkf([c0.spec(bb, refit_forgetting=0.8), c1.spec(bb)])
    n0, n1 = c0.G.n_nodes, c1.G.n_nodes
    X0 = np.concatenate([(c0.rng.standard_normal((n0, 32)) + 1.0).ravel(),
                         (c1.rng.standard_normal((n1, 24)) + 1.0).ravel()]).astype(np.float32)
    f.set_ensemble(_t(X0, np.float32))
    prev0 = np.asarray(X0[:n0 * 32], np.float64).reshape(n0, 32)
    V = np.concatenate([c0.noise().ravel(), c1.noise().ravel()])
    y = np.concatenate([c0.slopes(c0.truth()), c1.slopes(c1.truth())])
    f.step(_t(y, np.float32), V=_t(V, np.float32))
    torch.cuda.synchronize()
    got0 = f.get_ensemble().cpu().numpy().astype(np.float64)[:n0 * 32].reshape(n0, 32)
    rg = RF.ArRefit(0.97, 0.8)
    rg.update(got0.mean(axis=1), prev0.mean(axis=1))
    a, vs = f.get_model()
    assert abs(a[0] - rg.a) <= 1e-9 * rg.a and a[1] == 0.98 and vs[1] == 1.0
    # tuning runs frames but leaves the model (and the ensemble) as it was
    ens = f.get_ensemble().cpu().numpy()
    f.autotune(_t(y, np.float32), V=_t(V, np.float32), frames=2)
    assert np.array_equal(f.get_model()[0], a) and np.array_equal(f.get_ensemble().cpu().numpy(), ens)
    # a parameter change keeps the refitted model
    f.set_params(0, 1.1, 1.0, 0.0)
    assert np.array_equal(f.get_model()[0], a)
    f.reset_refit()
    a2, vs2 = f.get_model()
    assert a2[0] == 0.97 and vs2[0] == 1.0 and a2[1] == 0.98


def test_refit_refusals():
    bb = B()
    case = Case(8, None, 2, 1, 20, seed=67)
    for kw in ({"refit_forgetting": 1.5}, {"refit_forgetting": -0.1},
               {"refit_forgetting": 0.9, "ar2_coeff": 0.1}, {"refit_forgetting": 0.9, "ar_coeff": 1.0}):
        with pytest.raises(Exception):
            bb.Letkf([case.spec(bb, **kw)])
    g = bb.Letkf([case.spec(bb)])
    with pytest.raises(Exception):
        g.reset_refit()
    h = bb.Letkf([case.spec(bb, refit_forgetting=0.9)])
    xa = torch.zeros(h.sizes["ensemble_elems"], dtype=torch.float32, device=DEV)
    y = _t(case.slopes(case.truth()), np.float32)
    th = torch.zeros(3, dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        h.adjoint(xa, y, torch.zeros_like(xa), th, 0)
