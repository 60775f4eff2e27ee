"""Pins of the oracle's pre/post-processing (paper Sec. 3.5), reconstruction
through general per-mode operators (paper Sec. 8) and fixed-rank ST-HOSVD
(paper Sec. 9.4.1), against closed forms, invariants, brute force and the
already pinned subrange reconstruction.  CPU only."""
import itertools

import numpy as np
import pytest

import synthetic


def linear_index(dims):
    return np.arange(int(np.prod(dims)), dtype=np.float64)


@pytest.mark.parametrize("dims", [[3, 4, 3, 2], [5, 1, 7], [2, 9], [6]])
def test_slice_stats_closed_form_on_linear_index_tensor(orc, dims):
    """On the tensor whose element holds its own linear index (the paper's
    worked example of Sec. 4.2 is the 3x4x3x2 case), slice i of mode n holds
    e = l + L i + L J r for l < L, r < Rt: two independent uniform grids, so
    mean = L i + (L-1)/2 + L J (Rt-1)/2, variance = (L^2-1)/12 + (L J)^2 (Rt^2-1)/12,
    min = L i, max = L i + L-1 + L J (Rt-1), 1-norm = count * mean (all >= 0)
    and 2-norm^2 = count (variance + mean^2)."""
    X = linear_index(dims)
    for n in range(len(dims)):
        L = int(np.prod(dims[:n]))
        Rt = int(np.prod(dims[n + 1:]))
        J = dims[n]
        cnt = L * Rt
        st = orc.slice_stats(X, dims, n)
        i = np.arange(J)
        mean = L * i + (L - 1) / 2 + L * J * (Rt - 1) / 2
        var = (L * L - 1) / 12 + (L * J) ** 2 * (Rt * Rt - 1) / 12
        np.testing.assert_allclose(st[0], mean, rtol=1e-14)
        np.testing.assert_allclose(st[1], np.sqrt(var), rtol=1e-12, atol=1e-12)
        np.testing.assert_array_equal(st[2], L * i)
        np.testing.assert_array_equal(st[3], L * i + L - 1 + L * J * (Rt - 1))
        np.testing.assert_allclose(st[4], cnt * mean, rtol=1e-14)
        np.testing.assert_allclose(st[5], np.sqrt(cnt * (var + mean ** 2)), rtol=1e-13)


def test_slice_stats_signs_and_constant_slices(orc):
    """Negative values: the 1-norm sums magnitudes and min/max keep signs; a
    constant slice has standard deviation exactly 0, and its scale falls back
    to 1 in both pre-processing methods."""
    dims = [4, 3, 5]
    X = np.zeros(60)
    Xv = X.reshape(5, 3, 4)  # axes: mode 2, mode 1, mode 0
    Xv[:, 0, :] = -2.5       # slice 0 of mode 1: constant -2.5
    Xv[:, 1, :] = np.arange(20).reshape(5, 4) - 10.0
    Xv[:, 2, :] = 0.0        # slice 2: all zero
    st = orc.slice_stats(X, dims, 1)
    assert st[0][0] == -2.5 and st[1][0] == 0.0 and st[2][0] == -2.5 and st[3][0] == -2.5
    assert st[4][0] == 50.0 and st[5][0] == pytest.approx(np.sqrt(20 * 6.25), rel=1e-15)
    assert st[2][1] == -10.0 and st[3][1] == 9.0 and st[4][1] == 100.0
    assert st[0][2] == 0.0 and st[1][2] == 0.0 and st[5][2] == 0.0
    shift, scale = orc.scaling_vectors(st, "standardize")
    assert scale[0] == 1.0 and scale[2] == 1.0 and shift[0] == -2.5
    shift, scale = orc.scaling_vectors(st, "max")
    assert list(scale) == [2.5, 10.0, 1.0] and not shift.any()


@pytest.mark.parametrize("method", ["standardize", "max"])
def test_preprocessed_slices_are_normalised(orc, method):
    """After standardization every slice has mean 0 and standard deviation 1;
    after max rescaling every slice's largest magnitude is exactly 1 (the
    extreme value divided by itself)."""
    rng = np.random.default_rng(3)
    dims = [7, 5, 6, 4]
    X = rng.standard_normal(int(np.prod(dims))) * 3.0 + 11.0
    for n in range(4):
        st = orc.slice_stats(X, dims, n)
        shift, scale = orc.scaling_vectors(st, method)
        Z = orc.slice_transform(X, dims, n, shift, scale)
        st2 = orc.slice_stats(Z, dims, n)
        if method == "standardize":
            assert np.abs(st2[0]).max() <= 1e-14 * np.abs(st[0]).max() / st[1].min()
            np.testing.assert_allclose(st2[1], 1.0, rtol=1e-13)
        else:
            np.testing.assert_array_equal(np.maximum(np.abs(st2[2]), np.abs(st2[3])), 1.0)


def test_transform_inverse_round_trip(orc):
    rng = np.random.default_rng(4)
    dims = [6, 8, 3]
    X = rng.standard_normal(144) * 1e3
    shift = rng.standard_normal(8) * 10
    scale = rng.uniform(0.5, 4.0, 8)
    Z = orc.slice_transform(X, dims, 1, shift, scale)
    Xb = orc.slice_transform(Z, dims, 1, shift, scale, inverse=True)
    np.testing.assert_allclose(Xb, X, rtol=0, atol=4 * np.finfo(float).eps * np.abs(X).max())
    # the forward map is (x - shift_i) / scale_i along mode 1 (checked on one element)
    e = 5 + 6 * 3 + 48 * 2  # (l=5, i=3, r=2)
    assert Z[e] == (X[e] - shift[3]) / scale[3]


@pytest.fixture(scope="module")
def small_model(orc):
    X, dims = synthetic.random_tucker([9, 8, 7, 6], [3, 4, 2, 3], 1e-3, seed=12)
    return X, dims, orc.sthosvd(X, dims, 1e-4)


def test_range_operator_equals_subrange(orc, small_model):
    """A unit-step range operator is the half-open subrange of the already
    pinned reconstruction (selection is exact)."""
    X, dims, t = small_model
    b, e = [2, 0, 3, 1], [7, 8, 6, 4]
    Z, zd = orc.reconstruct_ops(t, [("range", bb, ee, 1) for bb, ee in zip(b, e)])
    Zs, zds = orc.reconstruct(t, b, e)
    assert zd == zds
    np.testing.assert_array_equal(Z, Zs)


def test_operators_against_bruteforce(orc, small_model):
    """Strided selection, averaging of consecutive indices (the paper's
    down-sampling example uses pairs), a sum and a mean, checked against loops
    over the brute-force reconstruction sum_r G[r] prod_n U_n[i_n, r_n]."""
    X, dims, t = small_model
    full = orc.reconstruct_bruteforce(t).reshape(dims[::-1])  # axes 3,2,1,0
    ops = [("average", 1, 9, 2), ("range", 0, 8, 3), ("sum", 2, 7), ("mean", 0, 6)]
    Z, zd = orc.reconstruct_ops(t, ops)
    assert zd == [4, 3, 1, 1]
    Z = Z.reshape(zd[::-1])
    for k0, k1 in itertools.product(range(4), range(3)):
        i0 = [1 + 2 * k0, 2 + 2 * k0]
        i1 = 3 * k1
        val = np.mean([full[:, 2:7, i1, a].sum(axis=1) for a in i0], axis=0).mean()
        assert Z[0, 0, k1, k0] == pytest.approx(val, rel=1e-12, abs=1e-14)


def test_sum_of_all_entries_closed_form(orc, small_model):
    """All-ones operators on every mode give sum_i X^[i] = sum_r G[r]
    prod_n (sum_i U_n[i, r_n]) (the paper's summary-statistic example with the
    count divided out gives the mean)."""
    X, dims, t = small_model
    Z, zd = orc.reconstruct_ops(t, [("sum", 0, d) for d in dims])
    G = t.core.reshape(t.ranks[::-1])
    colsums = [t.factors[n].sum(axis=0) for n in range(4)]
    closed = np.einsum("dcba,a,b,c,d->", G, *colsums)
    assert zd == [1, 1, 1, 1] and Z[0] == pytest.approx(closed, rel=1e-12)
    Zm, _ = orc.reconstruct_ops(t, [("mean", 0, d) for d in dims])
    assert Zm[0] == pytest.approx(closed / np.prod(dims), rel=1e-12)
    assert Zm[0] == pytest.approx(orc.reconstruct(t)[0].mean(), rel=1e-11)


def test_matrix_operator_is_applied_as_given(orc, small_model):
    X, dims, t = small_model
    rng = np.random.default_rng(5)
    Ct = rng.standard_normal((4, dims[2]))
    Z, zd = orc.reconstruct_ops(t, [None, None, ("matrix", Ct), None])
    full, _ = orc.reconstruct(t)
    ref = np.einsum("dcba,kc->dkba", full.reshape(dims[::-1]), Ct).reshape(-1)
    assert zd == [9, 8, 4, 6]
    np.testing.assert_allclose(Z, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("method", ["standardize", "max"])
def test_post_processing_inverts_pre_processing(orc, method):
    """Pre-process along the variable mode, compress with eps = 0 (nothing is
    discarded), reconstruct with the stored vectors: the original tensor comes
    back up to rounding; a per-variable mean through the operators equals the
    original data's."""
    X, dims, _ = synthetic.combustion((10, 9, 8, 5, 4), nbumps=6, seed=2)
    # give each variable (mode 3) its own scale and offset: C-order axes are (t, v, z, y, x)
    Xv = X.astype(np.float64).reshape(dims[::-1])
    Xv = Xv * np.array([1e-3, 1.0, 50.0, 2.0, 7.0])[None, :, None, None, None] + 3.0
    X = Xv.reshape(-1)
    st = orc.slice_stats(X, dims, 3)
    shift, scale = orc.scaling_vectors(st, method)
    Xp = orc.slice_transform(X, dims, 3, shift, scale)
    t = orc.sthosvd(Xp, dims, 0.0)
    Z, zd = orc.reconstruct_ops(t, post=(3, shift, scale))
    np.testing.assert_allclose(Z, X, rtol=0, atol=1e-10 * np.abs(X).max())
    v = 2
    Zm, _ = orc.reconstruct_ops(t, [("mean", 0, dims[0]), ("mean", 0, dims[1]), ("mean", 0, dims[2]),
                                    ("range", v, v + 1, 1), ("mean", 0, dims[4])], post=(3, shift, scale))
    assert Zm[0] == pytest.approx(st[0][v], rel=1e-10)


def test_fixed_rank_two_way_is_truncated_svd(orc):
    """N = 2 with given ranks (R, R): the Eckart-Young optimum, so the squared
    error is the sum of the dropped squared singular values."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 20)) @ np.diag(0.8 ** np.arange(20)) @ rng.standard_normal((20, 20))
    X = np.asfortranarray(A).reshape(-1, order="F")  # mode 0 fastest
    s = np.linalg.svd(A, compute_uv=False)
    for R in (1, 5, 12, 20):
        t = orc.sthosvd(X, [30, 20], 0.0, ranks=[R, R])
        assert t.ranks == [R, R]
        err2 = orc.relerr(X, t) ** 2 * orc.norm2(X)
        assert err2 == pytest.approx(np.sum(s[R:] ** 2), rel=1e-8, abs=1e-9 * s[0] ** 2)
        assert sum(t.discarded) == pytest.approx(err2, rel=1e-8, abs=1e-9 * s[0] ** 2)


def test_fixed_rank_recovers_low_rank_and_caps(orc):
    """Exact ranks of a noise-free Tucker tensor reproduce it; ranks above the
    mode sizes are capped at the current size; Corollary 1 holds."""
    X, dims = synthetic.random_tucker([12, 10, 8], [3, 4, 2], 0.0, seed=6)
    t = orc.sthosvd(X, dims, 0.5, ranks=[3, 4, 2])
    assert t.ranks == [3, 4, 2]
    assert orc.relerr(X, t) <= 1e-12
    t = orc.sthosvd(X, dims, 0.0, ranks=[50, 2, 50], order=[1, 0, 2])
    assert t.ranks == [12, 2, 8]
    e2 = orc.relerr(X, t) ** 2 * orc.norm2(X)
    assert sum(t.discarded) == pytest.approx(e2, rel=1e-9)
