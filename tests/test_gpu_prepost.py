"""GPU parity of the pre/post-processing subsystem (paper Sec. 3.5) and of
reconstruction through per-mode linear operators (paper Sec. 8), through the
C ABI, against the FP64 CPU oracle on the same inputs.

Tolerances, from the arithmetic:
* statistics: sums of n values in FP64 in a different order differ by at most
  about n u sum|x|: 1e-12 of the slice's 1-norm / count for the mean, and the
  same relative to the slice's 2-norm for the deviations; min and max exact.
* transform: the same FP64 expression ((x - s) / c, or fma(x, c, s)) rounded
  once, so bit-identical to the oracle given the same vectors.
* reconstruction: FP64 products in a different order, 1e-12 of the sum of
  |terms| (the oracle's reconstruction of |G| with |C_n^T| |U_n|).
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


def to_dev(x, dims, dtype):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(list(reversed(dims)))).to("cuda", dtype)


# row mapping (L >= 64), period mapping (L < 64, L*J <= 1024), the strided
# fallback (L < 64 with a long period: L = 1, J = 1500), ragged totals, N = 1
STAT_SHAPES = [
    ([70, 9, 13], [0, 1, 2]),
    ([3, 11, 400], [1]),
    ([1500, 7], [0]),
    ([5, 200, 3, 9], [0, 1, 2, 3]),
    ([1031], [0]),
    ([2, 3, 1, 5], [2]),
]


@pytest.mark.parametrize("dims,modes", STAT_SHAPES)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_slice_stats_parity(tk, orc, dims, modes, dtype):
    rng = np.random.default_rng(sum(dims))
    X = (rng.standard_normal(int(np.prod(dims))) * 2.0 + 5.0).astype(dtype)
    xd = to_dev(X, dims, torch.float64 if dtype == np.float64 else torch.float32)
    for n in modes:
        print(f"stats dims={dims} n={n} dtype={dtype.__name__}", flush=True)
        st = tk.slice_stats(xd, n, dims=dims).cpu().numpy()
        ref = orc.slice_stats(X.astype(np.float64), dims, n)
        cnt = X.size // dims[n]
        np.testing.assert_array_equal(st[2], ref[2])
        np.testing.assert_array_equal(st[3], ref[3])
        assert np.all(np.abs(st[0] - ref[0]) <= 1e-12 * ref[4] / cnt)
        assert np.all(np.abs(st[1] - ref[1]) <= 1e-12 * ref[5] / np.sqrt(cnt))
        np.testing.assert_allclose(st[4], ref[4], rtol=1e-12)
        np.testing.assert_allclose(st[5], ref[5], rtol=1e-12)


def test_slice_stats_large_mean_offset(tk, orc):
    """Data with |mean| >> std (a temperature-like field): the two-pass
    deviation sum keeps the standard deviation accurate."""
    dims = [64, 40, 6]
    rng = np.random.default_rng(5)
    X = 1.0e4 + rng.standard_normal(int(np.prod(dims)))
    st = tk.slice_stats(to_dev(X, dims, torch.float64), 2, dims=dims).cpu().numpy()
    ref = orc.slice_stats(X, dims, 2)
    np.testing.assert_allclose(st[1], ref[1], rtol=1e-9)


@pytest.mark.parametrize("method", ["standardize", "max"])
def test_scaling_vectors_match_oracle(tk, orc, method):
    rng = np.random.default_rng(2)
    stats = rng.standard_normal((6, 37))
    stats[1] = np.abs(stats[1])
    stats[1][[3, 8]] = 0.0
    stats[2][5], stats[3][5] = 0.0, 0.0
    sh, sc = tk.scaling_vectors(torch.from_numpy(stats).cuda(), method)
    rsh, rsc = orc.scaling_vectors(stats, method)
    np.testing.assert_array_equal(sh.cpu().numpy(), rsh)
    np.testing.assert_array_equal(sc.cpu().numpy(), rsc)


@pytest.mark.parametrize("dims,n", [([70, 9, 13], 1), ([3, 11, 401], 2), ([7], 0), ([5, 6, 7, 3], 0)])
@pytest.mark.parametrize("xdt,ydt", [(np.float64, np.float64), (np.float32, np.float32), (np.float32, np.float64),
                                     (np.float64, np.float32)])
def test_slice_transform_bit_exact(tk, orc, dims, n, xdt, ydt):
    rng = np.random.default_rng(sum(dims) + n)
    X = (rng.standard_normal(int(np.prod(dims))) * 30).astype(xdt)
    shift = rng.standard_normal(dims[n]) * 3
    scale = rng.uniform(0.2, 5.0, dims[n])
    tx = torch.float64 if xdt == np.float64 else torch.float32
    ty = torch.float64 if ydt == np.float64 else torch.float32
    xd = to_dev(X, dims, tx)
    sh, sc = torch.from_numpy(shift).cuda(), torch.from_numpy(scale).cuda()
    for inverse in (False, True):
        y = tk.slice_transform(xd, n, sh, sc, inverse=inverse, out_dtype=ty, dims=dims)
        ref = orc.slice_transform(X.astype(np.float64), dims, n, shift, scale, inverse=inverse).astype(ydt)
        np.testing.assert_array_equal(y.cpu().numpy().reshape(-1), ref)
    if xdt == ydt:  # in place
        y = xd.clone()
        tk.slice_transform(y, n, sh, sc, out=y, dims=dims)
        ref = orc.slice_transform(X.astype(np.float64), dims, n, shift, scale).astype(ydt)
        np.testing.assert_array_equal(y.cpu().numpy().reshape(-1), ref)


@pytest.fixture(scope="module")
def model(orc):
    """An oracle-made Tucker model, imported into a GPU handle."""
    X, dims = synthetic.random_tucker([23, 18, 11, 9], [5, 4, 3, 3], 1e-3, seed=44)
    return X, dims, orc.sthosvd(X, dims, 1e-4)


def _import(tk, t):
    core = torch.from_numpy(np.ascontiguousarray(t.core).reshape(t.ranks[::-1])).cuda()
    return tk.from_model(core, [torch.from_numpy(np.ascontiguousarray(U)).cuda() for U in t.factors])


def _abs_model(orc, t):
    return orc.Tucker(core=np.abs(t.core), factors=[np.abs(U) for U in t.factors], ranks=t.ranks, dims=t.dims,
                      eigenvalues=None, discarded=None, norm2=0.0, order=t.order)


def _abs_ops(ops, dims):
    out = []
    for op, d in zip(ops, dims):
        out.append(("matrix", np.abs(op[1])) if op is not None and op[0] == "matrix" else op)
    return out


OPS = [
    [None, None, None, None],
    [("range", 3, 20, 1), ("range", 0, 18, 4), None, ("range", 8, 9, 1)],
    [("average", 0, 23, 2), ("average", 1, 18, 3), ("range", 2, 3, 1), ("mean", 0, 9)],
    [("sum", 0, 23), ("sum", 0, 18), ("sum", 0, 11), ("sum", 0, 9)],
    [("mean", 5, 20), None, ("average", 0, 11, 11), ("range", 0, 9, 2)],
    [None, ("matrix", None), ("range", 1, 10, 3), None],
]


@pytest.mark.parametrize("case", range(len(OPS)))
@pytest.mark.parametrize("rule", ["flops", "memory"])
def test_reconstruct_ops_parity(tk, orc, model, case, rule):
    X, dims, t = model
    ops = list(OPS[case])
    rng = np.random.default_rng(case)
    dev_ops = []
    for n, op in enumerate(ops):
        if op is not None and op[0] == "matrix":
            Ct = rng.standard_normal((6, dims[n]))
            ops[n] = ("matrix", Ct)
            dev_ops.append(("matrix", torch.from_numpy(Ct).cuda()))
        else:
            dev_ops.append(op)
    g = _import(tk, t)
    Z = g.reconstruct_ops(dev_ops, rule=rule, out_dtype=torch.float64).cpu().numpy().reshape(-1)
    Zref, zd = orc.reconstruct_ops(t, ops)
    Aref, _ = orc.reconstruct_ops(_abs_model(orc, t), _abs_ops(ops, dims))
    assert Z.size == Zref.size
    assert np.all(np.abs(Z - Zref) <= 1e-12 * Aref + 1e-300), np.max(np.abs(Z - Zref) / (Aref + 1e-300))
    # float32 output: one more rounding of each value
    Z32 = g.reconstruct_ops(dev_ops, rule=rule, out_dtype=torch.float32).cpu().numpy().reshape(-1)
    assert np.all(np.abs(Z32 - Zref) <= 1e-12 * Aref + 2.0 ** -24 * np.abs(Zref) + 1e-300)
    g.free()


@pytest.mark.parametrize("method", ["standardize", "max"])
def test_postprocess_parity(tk, orc, model, method):
    """Post-processing of mode 2 (shift and scale, or scale only) through
    operators on every mode, including averaging and a mean on the
    post-processed mode, against the oracle's plain definition (reconstruct,
    undo the affine map, then apply the operators)."""
    X, dims, t = model
    rng = np.random.default_rng(9)
    shift = rng.standard_normal(dims[2]) * 4 if method == "standardize" else np.zeros(dims[2])
    scale = rng.uniform(0.5, 3.0, dims[2])
    g = _import(tk, t)
    g.set_postprocess(2, torch.from_numpy(shift).cuda() if method == "standardize" else None,
                      torch.from_numpy(scale).cuda())
    tabs = _abs_model(orc, t)
    for ops in ([None] * 4, [("range", 2, 9, 1), None, ("range", 4, 5, 1), ("range", 3, 9, 2)],
                [("mean", 0, 23), ("average", 0, 18, 2), ("average", 1, 11, 3), ("sum", 0, 9)],
                [None, None, ("mean", 0, 11), None]):
        Z = g.reconstruct_ops(ops, out_dtype=torch.float64).cpu().numpy().reshape(-1)
        Zref, _ = orc.reconstruct_ops(t, ops, post=(2, shift, scale))
        Aref, _ = orc.reconstruct_ops(tabs, ops, post=(2, np.abs(shift), scale))
        assert np.all(np.abs(Z - Zref) <= 1e-12 * Aref + 1e-300), np.max(np.abs(Z - Zref) / (Aref + 1e-300))
    # the plain subrange entry point applies it too
    Zs = g.reconstruct([1, 2, 3, 0], [20, 18, 8, 9], out_dtype=torch.float64).cpu().numpy().reshape(-1)
    Zref, _ = orc.reconstruct_ops(t, [("range", 1, 20, 1), ("range", 2, 18, 1), ("range", 3, 8, 1), None],
                                  post=(2, shift, scale))
    Aref, _ = orc.reconstruct_ops(tabs, [("range", 1, 20, 1), ("range", 2, 18, 1), ("range", 3, 8, 1), None],
                                  post=(2, np.abs(shift), scale))
    assert np.all(np.abs(Zs - Zref) <= 1e-12 * Aref + 1e-300)
    g.free()


@pytest.mark.parametrize("method", ["standardize", "max"])
def test_preprocess_compress_postprocess_round_trip(tk, orc, method):
    """The whole flow on a combustion-shaped float64 tensor with per-variable
    scales and offsets: pre-process the variable mode on the GPU, compress,
    attach the vectors, reconstruct; the relative error in the original
    units is at most eps * ||X'|| * max(scale) / ||X|| (the compression bound
    of the pre-processed tensor, mapped back), and with eps = 0 the original
    comes back to rounding."""
    X, dims, _ = synthetic.combustion((24, 20, 16, 5, 6), nbumps=8, seed=4)
    Xv = X.astype(np.float64).reshape(dims[::-1]) * np.array([1e-3, 1.0, 50.0, 2.0, 7.0])[None, :, None, None, None]
    X = (Xv + np.array([0.0, 300.0, -2.0, 1.0, 0.5])[None, :, None, None, None]).reshape(-1)
    x = to_dev(X, dims, torch.float64)
    y, shift, scale = tk.preprocess(x, 3, method)
    st = orc.slice_stats(X, dims, 3)
    rsh, rsc = orc.scaling_vectors(st, method)
    np.testing.assert_allclose(scale.cpu().numpy(), rsc, rtol=1e-10)
    np.testing.assert_allclose(shift.cpu().numpy(), rsh, rtol=1e-10, atol=1e-12 * np.abs(rsh).max())
    for eps in (0.0, 1e-3):
        t = tk.sthosvd(y, eps)
        t.set_postprocess(3, shift if method == "standardize" else None, scale)
        xh = t.reconstruct(out_dtype=torch.float64)
        err = float(torch.linalg.vector_norm((xh - x).reshape(-1)))
        nx = float(torch.linalg.vector_norm(x.reshape(-1)))
        ny = float(torch.linalg.vector_norm(y.reshape(-1)))
        if eps == 0.0:
            assert err <= 1e-12 * nx
        else:
            assert err <= eps * ny * float(scale.max()) * (1 + 1e-9)
        t.free()


def test_reconstruct_on_another_stream_then_free(tk, orc, model):
    """A reconstruction on a second stream, the handle freed right after, and
    new work on the owning stream: the result is intact."""
    X, dims, t = model
    g = _import(tk, t)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = g.reconstruct(out_dtype=torch.float64, stream=side)
    g.free()
    junk = [tk.sthosvd(torch.rand((9, 11, 18, 23), dtype=torch.float64, device="cuda"), 0.5) for _ in range(3)]
    side.synchronize()
    Zref, _ = orc.reconstruct(t)
    np.testing.assert_allclose(out.cpu().numpy().reshape(-1), Zref, rtol=0, atol=1e-12 * np.abs(Zref).max())
    del junk
