"""GPU parity: every step of the HIP path against the FP64 CPU oracle, called
through the C ABI (paper_1901_06043_amd is only argument marshalling).

Tolerances (FP64 path), derived from the arithmetic:
* Gram: a sum of K products in FP64 differs between summation orders by at most
  about K*u*sum|y_a||y_b|; we allow 1e-11 * sqrt(S_aa S_bb) per entry (K <= 1e6).
* Eigenvalues: backward-stable solvers agree to a few u*||S||*J; 1e-12*||S||.
* TTM: per entry 1e-12 * sum_j |M_kj||y_j|.
* Whole ST-HOSVD: identical ranks and |relerr_gpu - relerr_oracle| <= 1e-10
  (the acceptance bar of the method's FP64 path).
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


def to_dev(x, dims, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(list(reversed(dims)))).to("cuda", dtype)


GRAM_SHAPES = [
    ([64, 64, 64], [0, 1, 2]),
    ([200, 30, 7], [0, 1, 2]),
    ([16, 333, 5], [0, 1, 2]),
    ([11, 3, 40, 50], [0, 1, 2, 3]),
    ([130, 9, 3], [0, 1]),
    ([1, 7, 1, 5], [0, 1, 2, 3]),
    ([256, 65], [0, 1]),
    ([33, 2, 70], [0, 2]),
    ([232, 40], [0, 1]),   # 120 triangle blocks: the largest per-wave block count
    ([7, 232, 3], [1]),
    ([5], [0]),
    # the mode sizes of the 672x672x33x626 workload in the tile-pair kernel:
    # J = 672 with L = 1 (six 128-row tiles, 21 pairs, the last tile ragged),
    # J = 672 with L > 1, and J = 626 as the last mode (L > 1, no block above it)
    ([672, 1500], [0]),
    ([9, 672, 4], [1]),
    ([7, 5, 626], [2]),
    # FP64 Grams of J > 240: unit stride with even J (direct LDS loads) and a
    # ragged 44-row last tile; odd J and J = 999 over L = 301 columns (strides
    # not 16-byte aligned: register-staged tile pairs); L = 64 (direct loads,
    # five slabs); L = 447 (odd: register-staged); the last mode with
    # L = 1000; fewer columns than one chunk; L = 80 (a ragged chunk for float
    # input)
    ([300, 2000], [0]),
    ([301, 999], [0, 1]),
    ([64, 260, 5], [1]),
    ([447, 300, 3], [1]),
    ([1000, 250], [1]),
    ([300, 7], [0]),
    ([80, 384], [1]),
    # streaming Gram with the last row block's 1 or 2 rows on the VALU:
    # J = 17, 18, 34, 49 with unit stride, contiguous columns (L = 8) and
    # scalar loads (L = 3)
    ([17, 40, 9], [0]),
    ([8, 18, 30], [1]),
    ([3, 34, 20], [1]),
    ([49, 36], [0, 1]),
]


@pytest.mark.parametrize("dims,modes", GRAM_SHAPES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gram_parity(tk, orc, dims, modes, dtype):
    rng = np.random.default_rng(sum(dims))
    X = rng.standard_normal(int(np.prod(dims))).astype(dtype)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    Xd = to_dev(X, dims, tdt)
    for n in modes:
        print(f"gram dims={dims} n={n} dtype={dtype.__name__}", flush=True)
        S, nrm = tk.gram(Xd, n, dims=dims, with_norm=True)
        torch.cuda.synchronize()
        Sref = orc.gram(X.astype(np.float64), dims, n)
        d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref)))
        err = np.abs(S.cpu().numpy() - Sref)
        assert np.all(err <= 1e-11 * d + 1e-300), (err / (d + 1e-300)).max()
        assert float(nrm.item()) == pytest.approx(orc.norm2(X.astype(np.float64)), rel=1e-11)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gram_unaligned_base(tk, orc, dtype):
    """A tensor that starts one element past a 16-byte boundary: the FP64
    Gram of a large mode cannot use 16-byte direct loads and takes the
    register-staged tile-pair kernel."""
    dims = [260, 300]
    rng = np.random.default_rng(7)
    X = rng.standard_normal(int(np.prod(dims))).astype(dtype)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    buf = torch.empty(X.size + 4, dtype=tdt, device="cuda")
    x = buf[1:1 + X.size]
    x.copy_(torch.from_numpy(X))
    assert x.data_ptr() % 16 != 0
    x = x.view(dims[::-1])
    for n in (0, 1):
        print(f"gram unaligned dims={dims} n={n} dtype={dtype.__name__}", flush=True)
        S, nrm = tk.gram(x, n, dims=dims, with_norm=True)
        torch.cuda.synchronize()
        Sref = orc.gram(X.astype(np.float64), dims, n)
        d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref)))
        assert np.all(np.abs(S.cpu().numpy() - Sref) <= 1e-11 * d)
        assert float(nrm.item()) == pytest.approx(orc.norm2(X.astype(np.float64)), rel=1e-11)


def test_gram_large_columns_sampled(tk, orc):
    """Mode 0 of the 200x200x200x16 workload (K = 640000 columns): full Gram
    against the oracle on a column subset is impossible (the Gram sums all
    columns), so compare against the oracle Gram of the whole tensor."""
    X, dims = synthetic.decaying_200()
    Xd = to_dev(X, dims)
    S, nrm = tk.gram(Xd, 0, dims=dims, with_norm=True)
    Sref = orc.gram(X, dims, 0)
    d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref)))
    assert np.all(np.abs(S.cpu().numpy() - Sref) <= 1e-11 * d)
    assert float(nrm.item()) == pytest.approx(orc.norm2(X), rel=1e-11)


def _gram_of(rng, J, K, decay):
    A = rng.standard_normal((J, K)) * (decay ** np.arange(J))[:, None]
    return A @ A.T


# sizes on both sides of every register-phase boundary of the
# tridiagonalisation (32, 64, 96, 128, 192, 208) and the global-memory steps beyond
@pytest.mark.parametrize("J", [1, 2, 3, 11, 16, 32, 33, 50, 64, 65, 96, 97, 100, 128, 129, 192, 193, 200, 208, 209,
                               256, 300, 513, 672, 800, 1024])
def test_eig_truncate_parity(tk, orc, J):
    rng = np.random.default_rng(J)
    S = _gram_of(rng, J, J + 5, 0.8)
    nS = np.abs(np.linalg.eigvalsh(S)).max()
    for frac in (1e-1, 1e-4, 1e-9, 0.0):
        thr = frac * np.trace(S)
        lam, U, R, disc = tk.eig_truncate(torch.from_numpy(S).cuda(), thr)
        lref, Vref = orc.eig(S)
        Rref, dref = orc.truncate(lref, thr)
        lam = lam.cpu().numpy()
        U = U.cpu().numpy()
        assert np.abs(lam - lref).max() <= 1e-12 * nS
        # rank: equal to the oracle's unless the threshold falls within rounding
        # (64 u trace S) of a tail sum; then every rank on that tie is correct
        tail = np.concatenate([np.cumsum(np.clip(lref, 0, None)[::-1])[::-1], [0.0]])
        tol = 64 * np.finfo(float).eps * np.trace(S)
        ok = {r for r in range(1, J + 1) if tail[r] <= thr + tol and (r == 1 or tail[r - 1] >= thr - tol)}
        assert R == Rref or (R in ok and Rref in ok), (R, Rref, sorted(ok))
        assert disc == pytest.approx(tail[R], abs=tol + 1e-12 * nS)
        assert U.shape == (J, R)
        assert np.abs(U.T @ U - np.eye(R)).max() <= 1e-12
        assert np.linalg.norm(S @ U - U * lam[:R]) <= 1e-11 * nS
        # sign convention: in each column the largest-|entry| (lowest index) is positive
        for r in range(R):
            assert U[np.argmax(np.abs(U[:, r])), r] > 0
        # same vectors as the oracle where the eigenvalue is separated
        Uref = orc.sign_fix(Vref[:, :R])
        for r in range(R):
            gap = min([abs(lref[r] - lref[s]) for s in range(J) if s != r] or [nS])
            if gap > 1e-3 * nS:
                assert np.abs(U[:, r] - Uref[:, r]).max() <= 1e-9


def test_eig_repeated_eigenvalues(tk, orc):
    """Exactly repeated eigenvalues: any orthonormal basis of the eigenspace is
    correct; check residual, orthonormality and the eigenvalues."""
    J = 40
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((J, J)))
    lamt = np.array([5.0] * 4 + [2.0] * 6 + list(np.linspace(1, 0.01, J - 10)))
    S = (Q * lamt) @ Q.T
    S = (S + S.T) / 2
    lam, U, R, disc = tk.eig_truncate(torch.from_numpy(S).cuda(), 1e-3)
    lam, U = lam.cpu().numpy(), U.cpu().numpy()
    np.testing.assert_allclose(lam, np.sort(lamt)[::-1], atol=1e-12 * 5)
    assert np.abs(U.T @ U - np.eye(R)).max() <= 1e-12
    assert np.linalg.norm(S @ U - U * lam[:R]) <= 1e-11 * 5


TTM_CASES = [
    ([200, 50, 4], 0, 20),
    ([200, 50, 4], 1, 7),
    ([200, 50, 4], 2, 3),
    ([13, 17, 19], 1, 70),
    ([64, 64, 64], 2, 8),
    ([9, 5, 1, 3], 2, 4),
    ([100], 0, 130),
    # L = 1 with J = 2 mod 4 (paired-row loads) and odd J (single rows), for
    # the resident (K <= 64) and tiled kernels, with ragged last blocks
    ([102, 30], 0, 40),
    ([102, 30], 0, 70),
    ([101, 30], 0, 70),
    ([626, 9], 0, 130),
    # more than 64 output rows with direct LDS staging: L > 1 (L = 6: double
    # input only; L = 8 and 12: both; 128-column tiles crossing slabs of L),
    # the last mode (L = 200), ragged J and ragged row tiles (K = 130, 150)
    ([6, 100, 50], 1, 70),
    ([8, 90, 40], 1, 130),
    ([12, 40, 70], 1, 150),
    ([20, 10, 96], 2, 100),
    ([300, 50], 0, 260),
    # odd L or J with double input: 4-byte loads of Y
    ([9, 45, 33], 1, 150),
    ([99, 260], 0, 129),
    # FP64 resident products whose last row block holds one row (K = 17, 33,
    # 49; that row on the VALU): L = 1 with single, paired and 4-row loads,
    # and L > 1
    ([33, 40, 20], 0, 33),
    ([50, 30], 0, 49),
    ([64, 30], 0, 17),
    ([40, 33, 20], 1, 33),
]


@pytest.mark.parametrize("dims,n,K", TTM_CASES)
@pytest.mark.parametrize("ydt,zdt", [(np.float64, np.float64), (np.float32, np.float64), (np.float64, np.float32)])
def test_ttm_parity(tk, orc, dims, n, K, ydt, zdt):
    rng = np.random.default_rng(K + n)
    X = rng.standard_normal(int(np.prod(dims))).astype(ydt)
    M = rng.standard_normal((K, dims[n]))
    t_y = torch.float64 if ydt == np.float64 else torch.float32
    t_z = torch.float64 if zdt == np.float64 else torch.float32
    for Mview in (torch.from_numpy(M).cuda(), torch.from_numpy(np.asfortranarray(M)).cuda()):
        Z = tk.ttm(to_dev(X, dims, t_y), n, Mview, dims=dims, out_dtype=t_z)
        Zref, zd = orc.ttm(X.astype(np.float64), dims, n, M)
        Aref, _ = orc.ttm(np.abs(X.astype(np.float64)), dims, n, np.abs(M))
        tol = (1e-12 if zdt == np.float64 else 1e-6) * Aref + 1e-300
        assert np.all(np.abs(Z.cpu().numpy().reshape(-1).astype(np.float64) - Zref) <= tol)


@pytest.mark.parametrize("dims,n,K", TTM_CASES)
@pytest.mark.parametrize("ydt", [np.float64, np.float32])
def test_ttm_fp32_products_parity(tk, orc, dims, n, K, ydt):
    # products in FP32 (FP32 MFMA), accumulation in FP32: |error| <= J u32 |M||Y|
    rng = np.random.default_rng(3 * K + n)
    X = rng.standard_normal(int(np.prod(dims))).astype(ydt)
    M = rng.standard_normal((K, dims[n]))
    t_y = torch.float64 if ydt == np.float64 else torch.float32
    Z = tk.ttm(to_dev(X, dims, t_y), n, torch.from_numpy(M).cuda(), dims=dims, out_dtype=torch.float32,
               fp32_products=True)
    Zref, _ = orc.ttm(X.astype(np.float64), dims, n, M)
    Aref, _ = orc.ttm(np.abs(X.astype(np.float64)), dims, n, np.abs(M))
    tol = (dims[n] + 2) * 2.0 ** -23 * Aref + 1e-30
    assert np.all(np.abs(Z.cpu().numpy().reshape(-1).astype(np.float64) - Zref) <= tol)


@pytest.mark.parametrize("n", [0, 1])
def test_ttm_unaligned_base(tk, orc, n):
    """Double input starting 8 bytes past a 16-byte boundary: the tiled
    product loads Y in 4-byte pieces."""
    dims, K = [130, 90], 140
    rng = np.random.default_rng(11 + n)
    X = rng.standard_normal(int(np.prod(dims)))
    M = rng.standard_normal((K, dims[n]))
    buf = torch.empty(X.size + 2, dtype=torch.float64, device="cuda")
    x = buf[1:1 + X.size]
    x.copy_(torch.from_numpy(X))
    assert x.data_ptr() % 16 != 0
    print(f"ttm unaligned dims={dims} n={n}", flush=True)
    Z = tk.ttm(x.view(dims[::-1]), n, torch.from_numpy(M).cuda(), dims=dims, out_dtype=torch.float64)
    Zref, _ = orc.ttm(X, dims, n, M)
    Aref, _ = orc.ttm(np.abs(X), dims, n, np.abs(M))
    assert np.all(np.abs(Z.cpu().numpy().reshape(-1) - Zref) <= 1e-12 * Aref + 1e-300)


@pytest.mark.parametrize("order", [[0, 1, 2], [2, 0, 1]])
@pytest.mark.parametrize("given_ranks", [False, True])
def test_padded_working_extent(tk, orc, order, given_ranks):
    """An odd rank of mode 0 would leave mode 1 with an odd L: the working
    tensor carries a zero slice there (a zero column appended to U_0) and the
    core is compacted at the end.  Core and factors equal the oracle's up to
    column signs."""
    dims, ranks = [41, 30, 26], [5, 7, 6]
    X, dims = synthetic.random_tucker(dims, ranks, 1e-6, seed=21)
    print(f"padded extent order={order} given_ranks={given_ranks}", flush=True)
    x = to_dev(X, dims)
    if given_ranks:
        t = tk.sthosvd_ranks(x, ranks, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 0.0, order, ranks=ranks)
    else:
        t = tk.sthosvd(x, 1e-4, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 1e-4, order)
    assert t.ranks == ref.ranks == ranks
    G = t.core.cpu().numpy().reshape(-1)
    assert np.abs(np.abs(G) - np.abs(ref.core)).max() <= 1e-10 * np.abs(ref.core).max()
    for n in range(3):
        U = t.factor(n).cpu().numpy()
        Ur = ref.factors[n]
        sgn = np.sign(np.sum(U * Ur, axis=0))
        assert np.abs(U - Ur * sgn).max() <= 1e-9
    xh = t.reconstruct()
    e = float(torch.linalg.vector_norm((x - xh).reshape(-1)) / torch.linalg.vector_norm(x.reshape(-1)))
    assert abs(e - orc.relerr(X, ref)) <= 1e-10


@pytest.mark.parametrize("order", [[0, 1, 2, 3], [1, 0, 3, 2], [2, 1, 0, 3], [3, 2, 1, 0]])
@pytest.mark.parametrize("given_ranks", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_rank_mode_product_deferred(tk, orc, order, given_ranks, dtype):
    """Mode 1 keeps its full rank (R_1 = J_1 = 6): its product is a change of
    basis that leaves the later Grams unchanged, so it runs last, on the
    compact core (after the zero slice of the odd rank R_0 = 5 is dropped).
    Ranks, core and factors equal the oracle's up to column signs, and the
    error identity holds, in four orders (mode 1 first, in the middle and
    last), with eps and with given ranks, for float32 and float64 input."""
    dims, ranks = [41, 6, 26, 30], [5, 6, 7, 9]
    X, dims = synthetic.random_tucker(dims, ranks, 1e-6, seed=31)
    if dtype == torch.float32:
        X = X.astype(np.float32).astype(np.float64)
    print(f"deferred full-rank product order={order} given_ranks={given_ranks} dtype={dtype}", flush=True)
    x = to_dev(X, dims, dtype)
    if given_ranks:
        t = tk.sthosvd_ranks(x, ranks, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 0.0, order, ranks=ranks)
    else:
        t = tk.sthosvd(x, 1e-4, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 1e-4, order)
    assert t.ranks == ref.ranks == ranks
    G = t.core.cpu().numpy().reshape(-1)
    assert G.size == int(np.prod(ranks))
    Gs = G.reshape(ranks[::-1])
    Gr = ref.core.reshape(ranks[::-1])
    # the core up to the column signs of the factors
    sg = []
    for n in range(4):
        U = t.factor(n).cpu().numpy()
        Ur = ref.factors[n]
        sgn = np.sign(np.sum(U * Ur, axis=0))
        assert np.abs(U - Ur * sgn).max() <= 1e-9
        sg.append(sgn)
    S = np.einsum("a,b,c,d->dcba", sg[0], sg[1], sg[2], sg[3])
    assert np.abs(Gs - Gr * S).max() <= 1e-10 * np.abs(Gr).max()
    xh = t.reconstruct(out_dtype=torch.float64)
    e = float(torch.linalg.vector_norm((x.to(torch.float64) - xh).reshape(-1))
              / torch.linalg.vector_norm(x.to(torch.float64).reshape(-1)))
    assert abs(e - orc.relerr(X, ref)) <= 1e-10
    t.free()


@pytest.mark.parametrize("order", [[0, 1, 2], [1, 0, 2]])
@pytest.mark.parametrize("given_ranks", [False, True])
def test_padded_extent_compact_last_product(tk, orc, order, given_ranks):
    """The last mode has more than 64 rows of output, so its direct-load
    product writes the compact core itself, dropping the zero slice of the
    padded mode: mode 0 (order 0,1,2: the fastest mode) or mode 1 (order
    1,0,2: the zero slice sits between mode-0 rows).  Core and factors equal
    the oracle's up to column signs."""
    dims, ranks = [41, 30, 160], [9, 9, 70]
    X, dims = synthetic.random_tucker(dims, ranks, 1e-6, seed=23)
    print(f"compact last product order={order} given_ranks={given_ranks}", flush=True)
    x = to_dev(X, dims)
    if given_ranks:
        t = tk.sthosvd_ranks(x, ranks, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 0.0, order, ranks=ranks)
    else:
        t = tk.sthosvd(x, 1e-4, mode_order=order, dims=dims)
        ref = orc.sthosvd(X, dims, 1e-4, order)
    assert t.ranks == ref.ranks == ranks
    G = t.core.cpu().numpy().reshape(-1)
    assert G.size == int(np.prod(ranks))
    assert np.abs(np.abs(G) - np.abs(ref.core)).max() <= 1e-10 * np.abs(ref.core).max()
    for n in range(3):
        U = t.factor(n).cpu().numpy()
        Ur = ref.factors[n]
        sgn = np.sign(np.sum(U * Ur, axis=0))
        assert np.abs(U - Ur * sgn).max() <= 1e-9
    xh = t.reconstruct()
    e = float(torch.linalg.vector_norm((x - xh).reshape(-1)) / torch.linalg.vector_norm(x.reshape(-1)))
    assert abs(e - orc.relerr(X, ref)) <= 1e-10


def _check_sthosvd(tk, orc, X, dims, eps, order, dtype=torch.float64):
    print(f"sthosvd dims={dims} eps={eps} order={order}", flush=True)
    t = tk.sthosvd(to_dev(X, dims, dtype), eps, mode_order=order, dims=dims)
    ref = orc.sthosvd(X.astype(np.float64), dims, eps, order)
    assert t.ranks == ref.ranks
    assert t.norm2 == pytest.approx(ref.norm2, rel=1e-11)
    xh = t.reconstruct()
    x = to_dev(X, dims, torch.float64)
    e_gpu = float(torch.linalg.vector_norm((x - xh.to(torch.float64)).reshape(-1)) / torch.linalg.vector_norm(x.reshape(-1)))
    e_ref = orc.relerr(X.astype(np.float64), ref)
    assert abs(e_gpu - e_ref) <= 1e-10, (e_gpu, e_ref)
    assert e_gpu <= eps * (1 + 1e-9) + 1e-14
    # Corollary 1 on the GPU side: error^2 = sum of discarded eigenvalues
    assert abs(e_gpu ** 2 * t.norm2 - sum(t.discarded)) <= 1e-10 * t.norm2
    for n in range(len(dims)):
        U = t.factor(n).cpu().numpy()
        assert np.abs(U.T @ U - np.eye(t.ranks[n])).max() <= 1e-12
        np.testing.assert_allclose(t.eigenvalues(n).cpu().numpy(), ref.eigenvalues[n],
                                   atol=1e-12 * ref.eigenvalues[n][0])
    return t, ref


def test_sthosvd_lowrank_64(tk, orc):
    X, dims = synthetic.lowrank_64()
    t, ref = _check_sthosvd(tk, orc, X, dims, 1e-4, [0, 1, 2])
    assert t.ranks == [8, 8, 8]
    # separated spectra: factors and core agree with the oracle elementwise
    for n in range(3):
        np.testing.assert_allclose(t.factor(n).cpu().numpy(), ref.factors[n], atol=1e-9)
    G = t.core.cpu().numpy().reshape(-1)
    np.testing.assert_allclose(G, ref.core, atol=1e-9 * np.abs(ref.core).max())


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
@pytest.mark.parametrize("order", [[0, 1, 2, 3], [3, 2, 0, 1]])
def test_sthosvd_decaying_reduced(tk, orc, eps, order):
    X, dims = synthetic.decaying_200(scale=2)  # 100x100x100x16
    _check_sthosvd(tk, orc, X, dims, eps, order)


@pytest.mark.parametrize("case", [
    ([7, 1, 5], [2, 1, 2], 1e-2, 0.1),
    ([30], [3], 1e-3, 0.01),
    ([12, 9], [3, 2], 1e-3, 0.01),
    ([6, 5, 4, 3, 2], [2, 2, 2, 2, 2], 1e-2, 0.05),
    ([65, 17, 33], [5, 4, 3], 1e-3, 0.0),
])
def test_sthosvd_edge_shapes(tk, orc, case):
    dims, ranks, eta, eps = case
    X, dims = synthetic.random_tucker(dims, ranks, eta, seed=sum(dims))
    _check_sthosvd(tk, orc, X, dims, eps, None)


def test_sthosvd_float32_input(tk, orc):
    X, dims = synthetic.random_tucker([40, 30, 20], [4, 3, 2], 1e-3, seed=9, dtype=np.float32)
    _check_sthosvd(tk, orc, X, dims, 1e-2, [1, 0, 2], dtype=torch.float32)


def test_sthosvd_zero_tensor(tk):
    t = tk.sthosvd(torch.zeros((3, 4, 5), dtype=torch.float64, device="cuda"), 0.1)
    assert t.ranks == [1, 1, 1] and t.norm2 == 0.0


def test_sthosvd_nonfinite_rejected(tk):
    x = torch.zeros((3, 4, 5), dtype=torch.float64, device="cuda")
    x[1, 2, 3] = float("nan")
    with pytest.raises(tk.TuckerError) as ei:
        tk.sthosvd(x, 0.1)
    assert ei.value.name == "EINVAL"


def test_reconstruct_subrange_parity(tk, orc):
    X, dims = synthetic.decaying_200(scale=2)
    t = tk.sthosvd(to_dev(X, dims), 1e-4, dims=dims)
    ref = orc.sthosvd(X, dims, 1e-4)
    begin, end = [37, 37, 37, 0], [62, 62, 62, 16]
    for order in (None, [0, 1, 2, 3], [3, 1, 0, 2]):
        for odt in (torch.float64, torch.float32):
            Z = t.reconstruct(begin, end, order=order, out_dtype=odt)
            Zref, zd = orc.reconstruct(ref, begin, end)
            assert list(Z.shape) == zd[::-1]
            tol = 1e-9 if odt == torch.float64 else 1e-5
            np.testing.assert_allclose(Z.cpu().numpy().reshape(-1).astype(np.float64), Zref,
                                       atol=tol * np.abs(Zref).max())


@pytest.mark.parametrize("order", [[2, 0, 1], [1, 2, 0], [0, 1, 2]])
def test_reconstruct_odd_mode0_extent(tk, orc, order):
    """R_0 = 65 (odd): when mode 0 is not reconstructed first, the product just
    before it appends a zero slice to mode 0 (extent 66) and the mode-0
    product multiplies by the factor with a zero column appended, on 16-byte
    loads.  Full and sub-range reconstructions (an even and an odd number of
    mode-0 rows, where the latter keeps the odd extent), FP64 and FP32
    output, against the oracle's reconstruction."""
    dims, ranks = [130, 40, 96], [65, 20, 70]
    X, dims = synthetic.random_tucker(dims, ranks, 1e-6, seed=29)
    print(f"reconstruct odd mode-0 extent order={order}", flush=True)
    t = tk.sthosvd_ranks(to_dev(X, dims), ranks, dims=dims)
    ref = orc.sthosvd(X, dims, 0.0, ranks=ranks)
    assert t.ranks == ref.ranks == ranks
    for begin, end in (([0, 0, 0], dims), ([3, 5, 0], [127, 40, 96]), ([3, 0, 7], [126, 40, 90])):
        for odt in (torch.float64, torch.float32):
            Z = t.reconstruct(begin, end, order=order, out_dtype=odt)
            Zref, zd = orc.reconstruct(ref, begin, end)
            assert list(Z.shape) == zd[::-1]
            tol = 1e-9 if odt == torch.float64 else 1e-5
            np.testing.assert_allclose(Z.cpu().numpy().reshape(-1).astype(np.float64), Zref,
                                       atol=tol * np.abs(Zref).max())


def test_reconstruct_bad_range(tk):
    t = tk.sthosvd(torch.rand((4, 5, 6), dtype=torch.float64, device="cuda"), 0.1)
    with pytest.raises(tk.TuckerError):
        t.reconstruct([0, 0, 0], [7, 5, 4])
    with pytest.raises(tk.TuckerError):
        t.reconstruct([2, 0, 0], [2, 5, 4])


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_sthosvd_decaying_full_size(tk, orc, eps):
    """The 200x200x200x16 float64 workload at full size (the benchmark's)."""
    X, dims = synthetic.decaying_200()
    _check_sthosvd(tk, orc, X, dims, eps, [0, 1, 2, 3])


@pytest.mark.parametrize("case", [
    ([40, 30, 20], [5, 4, 3], [0, 1, 2], [40, 30, 20]),
    ([40, 30, 20], [5, 4, 3], [2, 0, 1], [3, 9, 2]),
    ([64, 64, 64], [8, 8, 8], [1, 2, 0], [8, 8, 8]),
    ([17, 1, 9, 6], [3, 1, 2, 2], [3, 0, 2, 1], [50, 1, 4, 50]),
    ([300, 20], [10, 8], [0, 1], [7, 7]),
])
def test_sthosvd_fixed_ranks_parity(tk, orc, case):
    """Fixed-rank ST-HOSVD (the core size is given): ranks min(R_n, J_n), the
    oracle's relative error within 1e-10, Corollary 1 on the GPU side,
    orthonormal factors and the oracle's eigenvalues."""
    dims, true_ranks, order, ranks = case
    X, dims = synthetic.random_tucker(dims, true_ranks, 1e-3, seed=sum(dims) + 3)
    print(f"fixed ranks dims={dims} ranks={ranks} order={order}", flush=True)
    t = tk.sthosvd_ranks(to_dev(X, dims), ranks, mode_order=order, dims=dims)
    ref = orc.sthosvd(X, dims, 0.0, order, ranks=ranks)
    assert t.ranks == ref.ranks
    x = to_dev(X, dims)
    xh = t.reconstruct()
    e_gpu = float(torch.linalg.vector_norm((x - xh).reshape(-1)) / torch.linalg.vector_norm(x.reshape(-1)))
    assert abs(e_gpu - orc.relerr(X, ref)) <= 1e-10
    assert abs(e_gpu ** 2 * t.norm2 - sum(t.discarded)) <= 1e-10 * t.norm2
    np.testing.assert_allclose(t.discarded, ref.discarded, rtol=1e-9, atol=1e-12 * ref.norm2)
    for n in range(len(dims)):
        U = t.factor(n).cpu().numpy()
        assert np.abs(U.T @ U - np.eye(t.ranks[n])).max() <= 1e-12
        np.testing.assert_allclose(t.eigenvalues(n).cpu().numpy(), ref.eigenvalues[n],
                                   atol=1e-12 * ref.eigenvalues[n][0])


def test_sthosvd_fixed_ranks_float32_and_reduced(tk, orc):
    X, dims = synthetic.random_tucker([60, 40, 30], [6, 5, 4], 1e-3, seed=77, dtype=np.float32)
    ref = orc.sthosvd(X.astype(np.float64), dims, 0.0, ranks=[6, 5, 4])
    t = tk.sthosvd_ranks(to_dev(X, dims, torch.float32), [6, 5, 4], dims=dims)
    assert t.ranks == [6, 5, 4] and t.core_dtype == tk.F64
    assert abs(np.sqrt(sum(t.discarded) / t.norm2) - orc.relerr(X.astype(np.float64), ref)) <= 1e-10
    t32 = tk.sthosvd_ranks(to_dev(X, dims, torch.float32), [6, 5, 4], prec="fp32", dims=dims)
    assert t32.ranks == [6, 5, 4] and t32.core_dtype == tk.F32
    xh = t32.reconstruct(out_dtype=torch.float64)
    x64 = to_dev(X, dims, torch.float64)
    e = float(torch.linalg.vector_norm((x64 - xh).reshape(-1)) / torch.linalg.vector_norm(x64.reshape(-1)))
    assert abs(e - orc.relerr(X.astype(np.float64), ref)) <= 1e-5
    # AUTO has no error target here and takes FP64
    ta = tk.sthosvd_ranks(to_dev(X, dims, torch.float32), [6, 5, 4], prec="auto", dims=dims)
    assert ta.gram_precision == ["fp64"] * 3
