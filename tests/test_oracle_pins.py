"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
formula: they check printed values (tests/golden), closed forms, identities,
textbook special cases (an SVD / eigvalsh from numpy as an independent
library routine) and brute force on tiny inputs.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_unfoldings():
    mats, cur = {}, None
    for line in open(os.path.join(GOLDEN, "unfoldings_3x4x3x2.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "mode":
            cur = int(tok[1])
            mats[cur] = {"rows": int(tok[2]), "cols": int(tok[3]), "data": []}
            continue
        mats[cur]["data"].append(tok)
    out = {}
    for n, m in mats.items():
        A = np.full((m["rows"], m["cols"]), np.nan)
        for i, tok in enumerate(m["data"]):
            if "..." in tok:
                k = tok.index("...")
                head, tail = tok[:k], tok[k + 1:]
                A[i, :len(head)] = [float(v) for v in head]
                A[i, m["cols"] - len(tail):] = [float(v) for v in tail]
            else:
                A[i, :] = [float(v) for v in tok]
        out[n] = A
    return out


EX_DIMS = [3, 4, 3, 2]
EX = np.arange(72, dtype=np.float64)  # entries equal their linear index (paper Fig. 1)


# ---------------------------------------------------------------- P1: unfolding

def test_unfold_matches_printed_example(orc):
    """Sec. 4.2: the printed unfoldings of the 3x4x3x2 linear-index tensor."""
    printed = _read_unfoldings()
    for n in range(4):
        U = orc.unfold(EX, EX_DIMS, n)
        P = printed[n]
        assert U.shape == P.shape
        mask = ~np.isnan(P)
        assert np.array_equal(U[mask], P[mask])


def test_gram_matches_printed_unfoldings(orc):
    """Alg. 2 on the worked example equals (printed unfolding)(printed unfolding)^T,
    exact integer arithmetic (modes 0-2 are printed in full)."""
    printed = _read_unfoldings()
    for n in range(3):
        P = printed[n]
        assert np.array_equal(orc.gram(EX, EX_DIMS, n), P @ P.T)
    # mode 3 is printed with elided columns: check the printed diagonal part
    S3 = orc.gram(EX, EX_DIMS, 3)
    P = printed[3]
    cols = ~np.isnan(P[0])
    part = P[:, cols] @ P[:, cols].T
    full = S3 - part
    # the 14 elided columns hold 12..25 and 48..61 (linear indices) by eq. idxtolin
    hid = np.array([np.arange(12, 26), np.arange(48, 62)], dtype=np.float64)
    assert np.array_equal(full, hid @ hid.T)


@pytest.mark.parametrize("dims", [[5], [7, 3], [3, 1, 4], [4, 5, 2, 3], [2, 3, 1, 2, 3], [1, 1, 6]])
def test_gram_general_shapes(orc, dims):
    """Gram of every mode equals unfold @ unfold.T (unfold is pinned by P1)."""
    rng = np.random.default_rng(11)
    Y = rng.standard_normal(int(np.prod(dims)))
    for n in range(len(dims)):
        U = orc.unfold(Y, dims, n)
        np.testing.assert_allclose(orc.gram(Y, dims, n), U @ U.T, rtol=1e-13, atol=1e-13)


def test_gram_thread_count_invariant(orc):
    rng = np.random.default_rng(3)
    dims = [9, 7, 5]
    Y = rng.standard_normal(int(np.prod(dims)))
    old = orc.NTHREADS
    try:
        orc.NTHREADS = 1
        a = orc.gram(Y, dims, 1)
        orc.NTHREADS = 5
        b = orc.gram(Y, dims, 1)
    finally:
        orc.NTHREADS = old
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- eigensolver

def test_eig_2x2_closed_form(orc):
    a, b, c = 3.0, -1.25, 0.5
    lam, V = orc.eig(np.array([[a, b], [b, c]]))
    m, d = (a + c) / 2, np.hypot((a - c) / 2, b)
    np.testing.assert_allclose(lam, [m + d, m - d], rtol=1e-15)
    S = np.array([[a, b], [b, c]])
    np.testing.assert_allclose(S @ V, V * lam, atol=1e-14)


def test_eig_diagonal_is_sorted_permutation(orc):
    d = np.array([0.5, 3.0, -1.0, 3.0, 2.0])
    lam, V = orc.eig(np.diag(d))
    assert list(lam) == [3.0, 3.0, 2.0, 0.5, -1.0]
    # stable: ties keep index order (index 1 before index 3)
    assert np.argmax(np.abs(V[:, 0])) == 1 and np.argmax(np.abs(V[:, 1])) == 3


@pytest.mark.parametrize("J", [3, 10, 37, 64])
def test_eig_known_spectrum(orc, J):
    """S = H diag(lam) H with a Householder reflector H: eigenvalues are lam."""
    rng = np.random.default_rng(J)
    v = rng.standard_normal(J)
    H = np.eye(J) - 2.0 * np.outer(v, v) / np.dot(v, v)
    lam_true = np.sort(rng.uniform(-2, 5, J))[::-1]
    S = (H * lam_true) @ H
    S = (S + S.T) / 2
    lam, V = orc.eig(S)
    np.testing.assert_allclose(lam, lam_true, atol=1e-13 * np.abs(lam_true).max())
    # eigenvectors are the columns of H up to sign
    np.testing.assert_allclose(np.abs(V.T @ H).max(axis=1), 1.0, atol=1e-10)


@pytest.mark.parametrize("J", [1, 2, 17, 50])
def test_eig_residual_orthogonality_and_library(orc, J):
    rng = np.random.default_rng(100 + J)
    A = rng.standard_normal((J, J + 3))
    S = A @ A.T  # a Gram matrix (PSD), as in the method
    lam, V = orc.eig(S)
    nS = np.linalg.norm(S)
    assert np.linalg.norm(S @ V - V * lam) <= 1e-13 * nS
    assert np.abs(V.T @ V - np.eye(J)).max() <= 1e-13
    np.testing.assert_allclose(lam, np.linalg.eigvalsh(S)[::-1], atol=1e-13 * nS)
    assert np.all(np.diff(lam) <= 0)


def test_eig_not_converged_flag(orc):
    with pytest.raises(orc.NotConverged):
        orc.eig(np.array([[1.0, 0.5], [0.5, 2.0]]), max_sweeps=0)


# ---------------------------------------------------------------- truncation (eq. Un)

@pytest.mark.parametrize("lam,thr,R,disc", [
    ([4, 3, 2, 1], 3.0, 2, 3.0),          # inclusive "<=" (tail of 2+1 == thr)
    ([4, 3, 2, 1], 2.999, 3, 1.0),
    ([4, 3, 2, 1], 0.0, 4, 0.0),          # nothing may be dropped
    ([4, 3, 2, 1], 100.0, 1, 6.0),        # R never below 1
    ([5, 0, 0], 0.0, 1, 0.0),
    ([5, 1, -1e-17], 0.0, 2, 0.0),        # negative round-off clamped to 0
    ([0, 0, 0], 0.0, 1, 0.0),             # zero tensor
    ([7], 0.0, 1, 0.0),
])
def test_truncate_cases(orc, lam, thr, R, disc):
    r, d = orc.truncate(np.array(lam, dtype=float), thr)
    assert (r, d) == (R, disc)


def test_sign_fix(orc):
    U = np.array([[0.1, 0.6, 0.5], [-0.9, 0.2, -0.5], [0.3, -0.7, 0.1]])
    F = orc.sign_fix(U)
    np.testing.assert_array_equal(F[:, 0], -U[:, 0])
    np.testing.assert_array_equal(F[:, 1], -U[:, 1])
    np.testing.assert_array_equal(F[:, 2], U[:, 2])  # tie 0.5 / -0.5: lowest row wins


# ---------------------------------------------------------------- TTM (Sec. 2.2.3)

@pytest.mark.parametrize("dims", [[6], [4, 5], [3, 4, 5], [2, 3, 4, 5], [3, 1, 2, 2, 3]])
def test_ttm_unfolding_identity(orc, dims):
    """Y x_n M  <=>  Z_(n) = M Y_(n) (unfold pinned by P1)."""
    rng = np.random.default_rng(7)
    Y = rng.standard_normal(int(np.prod(dims)))
    for n in range(len(dims)):
        for K in (1, 3, dims[n] + 2):
            M = rng.standard_normal((K, dims[n]))
            Z, zd = orc.ttm(Y, dims, n, M)
            assert zd[n] == K
            np.testing.assert_allclose(orc.unfold(Z, zd, n), M @ orc.unfold(Y, dims, n),
                                       rtol=1e-13, atol=1e-13)


def test_ttm_matches_tensordot(orc):
    rng = np.random.default_rng(8)
    dims = [3, 4, 5, 2]
    Y = rng.standard_normal(int(np.prod(dims)))
    T = Y.reshape(dims[::-1])
    for n in range(4):
        M = rng.standard_normal((6, dims[n]))
        ax = 3 - n
        ref = np.moveaxis(np.tensordot(M, T, axes=([1], [ax])), 0, ax).reshape(-1)
        Z, _ = orc.ttm(Y, dims, n, M)
        np.testing.assert_allclose(Z, ref, rtol=1e-13, atol=1e-13)


def test_ttm_commute_and_compose(orc):
    """Different modes commute; same mode composes as x_n V U (Sec. 2.2.3)."""
    rng = np.random.default_rng(9)
    dims = [4, 3, 5]
    Y = rng.standard_normal(60)
    A, B = rng.standard_normal((2, 4)), rng.standard_normal((6, 5))
    Z1, d1 = orc.ttm(*orc.ttm(Y, dims, 0, A), 2, B)
    Z2, d2 = orc.ttm(*orc.ttm(Y, dims, 2, B), 0, A)
    assert d1 == d2
    np.testing.assert_allclose(Z1, Z2, rtol=1e-13, atol=1e-13)
    U, V = rng.standard_normal((7, 3)), rng.standard_normal((2, 7))
    Z3, _ = orc.ttm(*orc.ttm(Y, dims, 1, U), 1, V)
    Z4, _ = orc.ttm(Y, dims, 1, V @ U)
    np.testing.assert_allclose(Z3, Z4, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- ST-HOSVD (Alg. 1)

CASES = [
    ([12, 10, 8], [3, 4, 2], 1e-3, 1e-1, [0, 1, 2]),
    ([9, 8, 7, 6], [3, 3, 2, 2], 1e-2, 5e-2, [2, 0, 3, 1]),
    ([6, 5, 4, 3, 2], [2, 2, 2, 2, 2], 1e-2, 1e-1, [4, 3, 2, 1, 0]),
    ([20, 15], [4, 3], 1e-3, 1e-2, [0, 1]),
    ([16, 16, 16], [5, 4, 3], 1e-4, 0.0, [0, 1, 2]),
    ([7, 9, 5], [2, 2, 2], 3e-1, 1e-1, [1, 2, 0]),
]


@pytest.mark.parametrize("dims,ranks,eta,eps,order", CASES)
def test_sthosvd_identities(orc, dims, ranks, eta, eps, order):
    """Cor. 1 (error = sum of discarded eigenvalues), the norm identity of Sec. 3,
    the eps guarantee of Alg. 1, orthonormal factors and rank caps."""
    import synthetic
    X, dims = synthetic.random_tucker(dims, ranks, eta, seed=sum(dims))
    t = orc.sthosvd(X, dims, eps, order)
    nx2 = orc.norm2(X)
    Xh, _ = orc.reconstruct(t)
    err2 = orc.norm2(X - Xh)
    assert abs(err2 - sum(t.discarded)) <= 1e-12 * nx2
    assert abs(err2 - (nx2 - orc.norm2(t.core))) <= 1e-12 * nx2
    assert np.sqrt(err2 / nx2) <= eps + 1e-12
    cur = list(dims)
    for n in order:
        U = t.factors[n]
        assert U.shape == (dims[n], t.ranks[n])
        assert np.abs(U.T @ U - np.eye(t.ranks[n])).max() <= 1e-12
        other = int(np.prod(cur)) // cur[n]
        assert 1 <= t.ranks[n] <= min(cur[n], other)
        assert len(t.eigenvalues[n]) == cur[n]
        cur[n] = t.ranks[n]


@pytest.mark.parametrize("dims,ranks,eta,eps,order", CASES)
def test_sthosvd_error_bounds(orc, dims, ranks, eta, eps, order):
    """Theorem 1 upper bound sum_n ||X x_n (I - U_n U_n^T)||^2 and the lower bound
    max_n sum_{i>R_n} sigma_i^2(X_(n)) (any rank-(R_n) Tucker model)."""
    import synthetic
    X, dims = synthetic.random_tucker(dims, ranks, eta, seed=sum(dims) + 1)
    t = orc.sthosvd(X, dims, eps, order)
    Xh, _ = orc.reconstruct(t)
    err2 = orc.norm2(X - Xh)
    nx2 = orc.norm2(X)
    upper, lower = 0.0, 0.0
    for n in range(len(dims)):
        U = t.factors[n]
        P = np.eye(dims[n]) - U @ U.T
        Z, _ = orc.ttm(X, dims, n, P)
        upper += orc.norm2(Z)
        s = np.linalg.svd(orc.unfold(X, dims, n), compute_uv=False)
        lower = max(lower, float(np.sum(s[t.ranks[n]:] ** 2)))
    assert err2 <= upper + 1e-12 * nx2
    assert err2 >= lower - 1e-12 * nx2


def test_first_mode_eigenvalues_are_squared_singular_values(orc):
    """Sec. 3.3: eigenvalues of X_(0) X_(0)^T are sigma^2 of X_(0) (numpy SVD)."""
    import synthetic
    X, dims = synthetic.random_tucker([11, 6, 5], [3, 3, 3], 1e-2, seed=5)
    for first in range(3):
        order = [first] + [m for m in range(3) if m != first]
        t = orc.sthosvd(X, dims, 1e-2, order)
        s = np.linalg.svd(orc.unfold(X, dims, first), compute_uv=False)
        ref = np.zeros(dims[first])
        ref[:len(s)] = s ** 2
        np.testing.assert_allclose(t.eigenvalues[first], ref, atol=1e-12 * orc.norm2(X))


@pytest.mark.parametrize("eps", [0.3, 0.05, 1e-3])
def test_two_way_is_truncated_svd(orc, eps):
    """N = 2: ST-HOSVD is a truncated SVD (Eckart-Young), checked against numpy."""
    rng = np.random.default_rng(21)
    I0, I1 = 13, 9
    A = rng.standard_normal((I0, 4)) @ rng.standard_normal((4, I1)) + 0.05 * rng.standard_normal((I0, I1))
    X = np.asfortranarray(A).reshape(-1, order="F")  # column-major: mode 0 fastest
    t = orc.sthosvd(X, [I0, I1], eps)
    Uf, s, Vt = np.linalg.svd(A)
    r = min(t.ranks)
    ref = (Uf[:, :r] * s[:r]) @ Vt[:r]
    Xh, _ = orc.reconstruct(t)
    np.testing.assert_allclose(Xh.reshape(I1, I0).T, ref, atol=1e-12 * s[0])
    assert np.sqrt(np.sum(s[r:] ** 2) / np.sum(s ** 2)) <= eps


def test_exact_low_rank_recovered(orc):
    """Sec. 9.2 generator with noise far below eps: ranks are the generator's."""
    import synthetic
    X, dims = synthetic.lowrank_64()
    t = orc.sthosvd(X, dims, 1e-4)
    assert t.ranks == [8, 8, 8]
    e = orc.relerr(X, t)
    assert 0.5e-6 < e < 1.0e-6 * 1.01


def test_zero_tensor_and_eps_zero(orc):
    t = orc.sthosvd(np.zeros(24), [2, 3, 4], 0.1)
    assert t.ranks == [1, 1, 1] and orc.norm2(t.core) == 0.0
    rng = np.random.default_rng(2)
    X = rng.standard_normal(24)
    t = orc.sthosvd(X, [2, 3, 4], 0.0)
    Xh, _ = orc.reconstruct(t)
    np.testing.assert_allclose(Xh, X, atol=1e-13)


def test_sthosvd_argument_errors(orc):
    X = np.zeros(6)
    with pytest.raises(ValueError):
        orc.sthosvd(X, [2, 3], -1.0)
    with pytest.raises(ValueError):
        orc.sthosvd(X, [2, 3], float("nan"))
    with pytest.raises(ValueError):
        orc.sthosvd(X, [2, 3], 0.1, [0, 0])
    with pytest.raises(ValueError):
        orc.sthosvd(X, [2, 4], 0.1)
    with pytest.raises(ValueError):
        orc.sthosvd(np.array([1.0, np.inf, 0, 0, 0, 0]), [2, 3], 0.1)


# ---------------------------------------------------------------- reconstruction (Sec. 8)

def test_reconstruct_matches_bruteforce_and_any_order(orc):
    """Multi-TTM over index sub-ranges equals the explicit sum over the core, and
    every TTM order gives the same result (Sec. 8)."""
    import synthetic
    X, dims = synthetic.random_tucker([5, 4, 3, 4], [2, 3, 2, 2], 0.05, seed=3)
    t = orc.sthosvd(X, dims, 0.05)
    begin, end = [1, 0, 1, 2], [4, 3, 3, 4]
    ref = orc.reconstruct_bruteforce(t, begin, end)
    for order in itertools.permutations(range(4)):
        Z, zd = orc.reconstruct(t, begin, end, list(order))
        assert zd == [3, 3, 2, 2]
        np.testing.assert_allclose(Z, ref, rtol=1e-13, atol=1e-13)


def test_full_reconstruct_bruteforce(orc):
    import synthetic
    X, dims = synthetic.random_tucker([4, 3, 5], [2, 2, 3], 0.01, seed=4)
    t = orc.sthosvd(X, dims, 1e-2)
    Z, _ = orc.reconstruct(t)
    np.testing.assert_allclose(Z, orc.reconstruct_bruteforce(t), rtol=1e-13, atol=1e-13)
