"""Modes above 1024 (up to the eigensolver's 2304): one GPU's share of the
paper's larger grids has modes of 1500 and 2080 (Sec. 9.2).  At these sizes
the oracle's Jacobi eigensolver takes minutes, so the eigensolver is pinned by
matrices of known spectrum (S = Q diag(lam) Q^T, Weyl's bound) and the whole
compression by properties that hold at any size: exact ranks of a low-rank
tensor, orthonormal factors, the error identity of Cor. 1 and the eps bound,
with the Gram checked entry by entry against the oracle's Gram and its
eigenvalues against numpy's LAPACK solver.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_1901_06043_amd as tk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tk.lib()
    return tk


def _known_spectrum(J, seed):
    """S = Q diag(lam) Q^T: a decaying head, then a dense cluster (all within
    1e-2 of the largest, so the kept vectors are re-orthogonalised as one
    window), then a few exact zeros."""
    rng = np.random.default_rng(seed)
    Q, Rq = np.linalg.qr(rng.standard_normal((J, J)))
    Q = Q * np.sign(np.diag(Rq))
    head = 0.7 ** np.arange(40)
    cluster = 1e-4 * (1.0 + 0.5 * rng.random(J - 48))
    lam = np.concatenate([head, cluster, np.zeros(8)])
    S = (Q * lam) @ Q.T
    return (S + S.T) / 2, np.sort(lam)[::-1], Q, lam


@pytest.mark.parametrize("J", [1025, 1500, 2080, 2304])
def test_eig_large_known_spectrum(tk, J):
    print(f"eig large J={J}", flush=True)
    S, lam_true, Q, lam_unsorted = _known_spectrum(J, J)
    nS = 1.0
    for frac in (1e-1, 1e-6):  # a handful of vectors, then nearly all of them
        thr = frac * np.trace(S)
        lam, U, R, disc = tk.eig_truncate(torch.from_numpy(S).cuda(), thr)
        lam = lam.cpu().numpy()
        U = U.cpu().numpy()
        # Weyl: forming S in FP64 moves each eigenvalue by at most ~J u ||S||
        assert np.abs(lam - lam_true).max() <= 1e-12 * nS
        # truncation rule (eq. Un) on the returned eigenvalues
        tail = np.concatenate([np.cumsum(np.clip(lam, 0, None)[::-1])[::-1], [0.0]])
        assert tail[R] <= thr and (R == 1 or tail[R - 1] > thr)
        assert disc == pytest.approx(tail[R], abs=64 * np.finfo(float).eps * np.trace(S))
        assert U.shape == (J, R)
        assert np.abs(U.T @ U - np.eye(R)).max() <= 1e-12
        assert np.linalg.norm(S @ U - U * lam[:R]) <= 1e-11 * nS * np.sqrt(R)
        for r in range(R):
            assert U[np.argmax(np.abs(U[:, r])), r] > 0
        # the head above the cluster (gaps >= 2.4e-4): the known eigenvectors
        # up to sign, within about J u ||S|| / gap
        order = np.argsort(-lam_unsorted, kind="stable")
        for r in range(min(R, 20)):
            q = Q[:, order[r]]
            q = q * np.sign(q[np.argmax(np.abs(q))])
            assert np.abs(U[:, r] - q).max() <= 1e-8


@pytest.mark.parametrize("dims,ranks,order", [
    ([2080, 24, 20], [12, 6, 5], [0, 1, 2]),
    ([20, 1500, 24], [5, 14, 6], [2, 1, 0]),
])
def test_sthosvd_large_mode_exact_ranks(tk, orc, dims, ranks, order):
    """A Tucker tensor of known ranks plus 1e-9 noise: eps = 1e-6 recovers the
    ranks exactly (P8), with orthonormal factors and the error identity."""
    print(f"sthosvd large mode dims={dims} ranks={ranks} order={order}", flush=True)
    X, dims = synthetic.random_tucker(dims, ranks, 1e-9, seed=sum(dims))
    x = torch.from_numpy(X.reshape(dims[::-1])).cuda()
    eps = 1e-6
    t = tk.sthosvd(x, eps, mode_order=order)
    assert list(t.ranks) == ranks
    nx2 = orc.norm2(X)
    assert t.norm2 == pytest.approx(nx2, rel=1e-12)
    for n in range(3):
        U = t.factor(n).cpu().numpy()
        assert np.abs(U.T @ U - np.eye(ranks[n])).max() <= 1e-12
    Xh = t.reconstruct().cpu().numpy().reshape(-1)
    rel = np.linalg.norm(X - Xh) / np.sqrt(nx2)
    assert rel <= eps
    # Cor. 1: the squared error is the discarded energy; here both are at the
    # rounding level of the eigenvalues (about J u ||X||^2 in all)
    assert abs(rel ** 2 - sum(t.discarded) / nx2) <= 1e-11
    t.free()


def test_sthosvd_large_mode_noise(tk, orc):
    """Gaussian noise of 1500 x 40 x 30: at eps = 0.3 the mode-0 rank is large
    (several hundred kept vectors, whose blocks are re-orthogonalised in place
    in global memory).  The mode-0 Gram matches the oracle's entry by entry, its
    eigenvalues match LAPACK's, and the result keeps the eps bound, the error
    identity and orthonormal factors."""
    dims = [1500, 40, 30]
    rng = np.random.default_rng(1500)
    X = rng.standard_normal(int(np.prod(dims)))
    x = torch.from_numpy(X.reshape(dims[::-1])).cuda()
    print("gram J=1500 vs oracle", flush=True)
    S = tk.gram(x, 0, dims=dims).cpu().numpy()
    Sref = orc.gram(X, dims, 0)
    d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref)))
    assert np.all(np.abs(S - Sref) <= 1e-11 * d)
    lam_ref = np.linalg.eigvalsh(Sref)[::-1]
    eps = 0.3
    print("sthosvd J=1500 noise", flush=True)
    t = tk.sthosvd(x, eps, mode_order=[0, 1, 2])
    nx2 = orc.norm2(X)
    lam = t.eigenvalues(0).cpu().numpy()
    assert np.abs(lam - lam_ref).max() <= 1e-12 * lam_ref[0]
    R0 = t.ranks[0]
    assert R0 > 300
    thr = eps ** 2 * nx2 / 3
    tail = np.concatenate([np.cumsum(np.clip(lam, 0, None)[::-1])[::-1], [0.0]])
    assert tail[R0] <= thr and tail[R0 - 1] > thr
    for n in range(3):
        U = t.factor(n).cpu().numpy()
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-12
    U0 = t.factor(0).cpu().numpy()
    assert np.linalg.norm(Sref @ U0 - U0 * lam[:R0]) <= 1e-11 * lam_ref[0] * np.sqrt(R0)
    Xh = t.reconstruct().cpu().numpy().reshape(-1)
    rel = np.linalg.norm(X - Xh) / np.sqrt(nx2)
    assert rel <= eps
    assert abs(rel ** 2 - sum(t.discarded) / nx2) <= 1e-10
    t.free()


def test_mode_above_eigensolver_limit(tk):
    """A mode of 2305 is refused before any work (EUNSUPPORTED)."""
    x = torch.zeros(2, 2, 2305, dtype=torch.float64, device="cuda")
    with pytest.raises(tk.TuckerError) as e:
        tk.sthosvd(x, 1e-3)
    assert e.value.status == 5
    assert "2304" in str(e.value)
