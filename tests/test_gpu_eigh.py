"""The FP64 wave-level eigensolve alone against LAPACK (numpy.linalg.eigh)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _spd(rng, batch, m, p, c):
    Y = rng.standard_normal((batch, p, m)) * rng.uniform(0.5, 20, (batch, 1, 1))
    Y -= Y.mean(axis=2, keepdims=True)   # anomalies: 1 is an eigenvector, eigenvalue c
    return c * np.eye(m) + np.einsum("bpi,bpj->bij", Y, Y)


@pytest.mark.parametrize("m,p", [(64, 72), (64, 20), (50, 50), (20, 32), (2, 8), (33, 4)])
def test_eigh_matches_lapack(m, p):
    from paper_1408_7069_amd import binding as B
    rng = np.random.default_rng(m * 100 + p)
    A = _spd(rng, 12, m, p, (m - 1) / 1.05)
    Q, lam, sw = B.eigh_spd(torch.from_numpy(A).cuda(), tol=1e-14, max_sweeps=40)
    Q, lam, sw = Q.cpu().numpy(), lam.cpu().numpy(), sw.cpu().numpy()
    assert np.all(sw > 0), sw
    for k in range(A.shape[0]):
        nA = np.linalg.norm(A[k], 2)
        assert np.linalg.norm(A[k] @ Q[k] - Q[k] * lam[k], 2) <= 1e-12 * nA
        assert np.linalg.norm(Q[k].T @ Q[k] - np.eye(m), 2) <= 1e-13
        ref = np.linalg.eigvalsh(A[k])
        assert np.abs(np.sort(lam[k]) - ref).max() <= 1e-12 * ref.max()


def test_eigh_nonconvergence_is_reported():
    from paper_1408_7069_amd import binding as B
    rng = np.random.default_rng(3)
    A = _spd(rng, 4, 64, 72, 60.0)
    _, _, sw = B.eigh_spd(torch.from_numpy(A).cuda(), tol=1e-14, max_sweeps=1)
    assert np.all(sw.cpu().numpy() == -1)
