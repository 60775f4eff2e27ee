"""GPU checks of the reduced-precision forms (FP32-MFMA, BF16x3 and BF16x6
Grams; FP32 working tensor with FP32-MFMA mode products) through the C ABI,
against the FP64 CPU oracle on the same float32 data.

Per-entry Gram bounds, from the arithmetic (d_ab = sqrt(S_aa S_bb), which
bounds sum_k |y_ak y_bk| by Cauchy-Schwarz; u = 2^-24):
* FP32: one 32-column chunk is summed in FP32 (8 MFMA steps), then added in
  FP64: |err| <= (32 + 8) u d_ab = 2.4e-6 d_ab.
* BF16X3: per product the dropped pieces b1 c1, (b0 + b1) s and r (c0 + c1)
  are each at most 2^-16 |x y| (1 + 2^-7), and a group of 8 chunks accumulates
  3 * 256 products in FP32: (768 + 8) u + 3.1 * 2^-16 = 9.4e-5.
* BF16X6: the dropped pieces are O(2^-24) and a chunk accumulates 6 * 32
  products in FP32: (192 + 14) u = 1.2e-5.
The typical (root-mean-square) error is far below these worst cases; it is
checked too, so that a lost product term (error ~2^-8) cannot hide.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
BOUND = {"fp32": (32 + 8) * U32, "bf16x3": (768 + 8) * U32 + 3.1 * 2.0 ** -16, "bf16x6": (192 + 14) * U32}
RMS = {"fp32": 3e-7, "bf16x3": 2e-5, "bf16x6": 3e-7}


@pytest.fixture(scope="module")
def tk():
    import paper_1901_06043_amd as tk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tk.lib()
    return tk


def to_dev(x, dims, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x).reshape(list(reversed(dims)))).to("cuda", dtype)


MP_SHAPES = [
    ([64, 64, 64], [0, 1, 2]),
    ([200, 30, 7], [0, 1, 2]),
    ([16, 333, 5], [0, 1, 2]),
    ([11, 3, 40, 50], [0, 1, 2, 3]),
    ([130, 9, 3], [0, 1]),
    ([1, 7, 1, 5], [0, 1, 2, 3]),
    ([256, 65], [0, 1]),
    ([128, 300], [0, 1]),
    ([520, 40], [0]),  # L = 1 pair mode with five row tiles, the last one ragged
    ([5], [0]),
    ([672, 600], [0]),  # the 672x672x33x626 workload's mode sizes: six and five row tiles
    ([9, 672, 3], [1]),
    ([7, 5, 626], [2]),
]


@pytest.mark.parametrize("dims,modes", MP_SHAPES)
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16x6"])
def test_gram_reduced_parity(tk, orc, dims, modes, prec):
    rng = np.random.default_rng(sum(dims) + 7)
    X = rng.standard_normal(int(np.prod(dims))).astype(np.float32)
    Xd = to_dev(X, dims)
    for n in modes:
        print(f"gram {prec} dims={dims} n={n}", flush=True)
        S, nrm = tk.gram(Xd, n, prec=prec, dims=dims, with_norm=True)
        Sref = orc.gram(X.astype(np.float64), dims, n)
        d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref))) + 1e-300
        rel = np.abs(S.cpu().numpy() - Sref) / d
        assert rel.max() <= BOUND[prec], rel.max()
        assert np.sqrt(np.mean(rel ** 2)) <= RMS[prec], np.sqrt(np.mean(rel ** 2))
        # the sum of squares is FP64 whatever the Gram arithmetic
        assert float(nrm.item()) == pytest.approx(orc.norm2(X.astype(np.float64)), rel=1e-11)


@pytest.mark.parametrize("dims", [[48, 4000], [256, 600]])
def test_bf16x3_bias_bf16x6_unbiased(tk, orc, dims):
    """The product dropped by BF16X3 is a Gram of bf16 rounding residuals, so
    its trace error is negative and about 2^-16/3 of the trace (uniform
    residuals); BF16X6 removes it.  A mode of 48 takes the streaming kernel,
    one of 256 the tile pairs (BF16X6: with direct loads)."""
    rng = np.random.default_rng(11)
    X = rng.standard_normal(int(np.prod(dims))).astype(np.float32)
    Sref = orc.gram(X.astype(np.float64), dims, 0)
    tr = np.trace(Sref)
    d3 = np.trace(tk.gram(to_dev(X, dims), 0, prec="bf16x3", dims=dims).cpu().numpy()) - tr
    d6 = np.trace(tk.gram(to_dev(X, dims), 0, prec="bf16x6", dims=dims).cpu().numpy()) - tr
    assert -3e-5 * tr < d3 < -2e-6 * tr, d3 / tr
    assert abs(d6) < 1e-6 * tr, d6 / tr


@pytest.mark.parametrize("dims,n,K", [([200, 50, 4], 0, 20), ([13, 17, 19], 1, 70), ([64, 64, 64], 2, 8),
                                      ([300, 40], 0, 130)])
def test_ttm_fp32_products(tk, orc, dims, n, K):
    rng = np.random.default_rng(K + n + 1)
    X = rng.standard_normal(int(np.prod(dims))).astype(np.float32)
    M = rng.standard_normal((K, dims[n]))
    Z = tk.ttm(to_dev(X, dims), n, torch.from_numpy(M).cuda(), dims=dims, out_dtype=torch.float32,
               fp32_products=True)
    Zref, _ = orc.ttm(X.astype(np.float64), dims, n, M)
    Aref, _ = orc.ttm(np.abs(X.astype(np.float64)), dims, n, np.abs(M))
    J = dims[n]
    tol = (J + 4) * U32 * Aref + U32 * np.abs(Zref) + 1e-300
    err = np.abs(Z.cpu().numpy().reshape(-1).astype(np.float64) - Zref)
    assert np.all(err <= tol), (err / tol).max()
    # and FP32 products are not FP64 ones: a few entries must differ from an FP64-product TTM
    Z64 = tk.ttm(to_dev(X, dims), n, torch.from_numpy(M).cuda(), dims=dims, out_dtype=torch.float64)
    assert np.abs(Z64.cpu().numpy().reshape(-1) - Zref).max() <= 1e-12 * Aref.max()


@pytest.mark.parametrize("scale,prec", [(1e20, "fp32"), (1e-25, "fp32"), (1e20, "bf16x3"), (1e-25, "bf16x6")])
def test_range_handling_scales_slices(tk, orc, scale, prec):
    """FP32 squares overflow above ~1.8e19 and vanish below ~1e-23: the guard
    sees the trace, a non-finite entry or a diagonal outside the safe range,
    and the Gram is redone in the same reduced form on the per-slice scaled
    copy (powers of two), so the result equals the FP64 oracle's ranks."""
    X, dims = synthetic.random_tucker([30, 20, 10], [4, 3, 2], 1e-3, seed=21)
    X = (X * scale).astype(np.float32)
    t = tk.sthosvd(to_dev(X, dims), 1e-2, prec=prec, dims=dims)
    ref = orc.sthosvd(X.astype(np.float64), dims, 1e-2)
    assert t.gram_precision[0] == prec and t.gram_scaled[0]
    assert t.ranks == ref.ranks
    assert t.norm2 == pytest.approx(ref.norm2, rel=1e-11)
    # in range: no second pass
    Xn = (X.astype(np.float64) / scale).astype(np.float32)
    t2 = tk.sthosvd(to_dev(Xn, dims), 1e-2, prec=prec, dims=dims)
    assert t2.gram_precision == [prec] * 3 and not any(t2.gram_scaled)


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_per_slice_scaling_small_magnitudes(tk, orc, prec):
    """Slices of mode 0 with magnitudes 1e-24 .. 1e-22: their squares lie below
    the FP32 normal range, so the plain reduced Gram loses them; the guard sees
    the diagonal out of range and the scaled pass computes the Gram to the
    form's accuracy, so every eigenvalue is within Weyl's bound
    ||E||_2 <= bound * trace S of the oracle's."""
    rng = np.random.default_rng(3)
    dims = [12, 40, 30]
    X = rng.standard_normal(int(np.prod(dims))).reshape(30, 40, 12)
    X *= (10.0 ** rng.uniform(-24, -22, 12))[None, None, :]
    X = X.astype(np.float32).reshape(-1)
    t = tk.sthosvd(to_dev(X, dims), 1e-2, prec=prec, dims=dims)
    assert t.gram_scaled[0] and t.gram_precision[0] == prec
    lam = t.eigenvalues(0).cpu().numpy()
    lref, _ = orc.eig(orc.gram(X.astype(np.float64), dims, 0))
    tr = float(np.sum(lref))
    assert np.abs(lam - lref).max() <= (BOUND[prec] + 64 * 2.0 ** -52) * tr


@pytest.mark.parametrize("eps,want", [(1e-3, "fp64"), (3e-2, "fp32"), (0.2, "bf16x3")])
def test_auto_precision_rule(tk, orc, eps, want):
    """AUTO takes the cheapest form whose predicted error (2^-16/3 of ||X||^2
    for BF16X3, 2^-23 for FP32) is within 1% of the slack of the 1.05 eps
    target, (1.05^2 - 1) eps^2 ||X||^2 / N (N = 3: FP32 from eps = 0.0187,
    BF16X3 from 0.122), and FP64 otherwise; FP64 data always takes FP64."""
    X, dims = synthetic.random_tucker([40, 30, 20], [6, 5, 4], 1e-2, seed=5, dtype=np.float32)
    t = tk.sthosvd(to_dev(X, dims), eps, prec="auto", dims=dims)
    assert t.gram_precision == [want] * 3
    assert t.core_dtype == (tk.F64 if want == "fp64" else tk.F32)
    ref = orc.sthosvd(X.astype(np.float64), dims, eps)
    xh = t.reconstruct(out_dtype=torch.float64)
    x64 = to_dev(X, dims).double()
    e = float(torch.linalg.vector_norm((x64 - xh).reshape(-1)) / torch.linalg.vector_norm(x64.reshape(-1)))
    assert e <= 1.05 * eps
    assert t.ranks == ref.ranks
    t64 = tk.sthosvd(to_dev(X, dims, torch.float64), eps, prec="auto", dims=dims)
    assert t64.gram_precision == ["fp64"] * 3


def _principal_sin(Ua, Ub):
    """Largest principal angle sine between the column spaces of Ua and Ub."""
    s = np.linalg.svd(Ua.T @ Ub, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def _mixed_report(tk, orc, X, dims, eps, order, prec):
    """Compress with a reduced form and compare with the FP64 oracle: ranks,
    relative error (explicit FP64 reconstruction on the GPU), per-mode largest
    principal angle (where ranks agree), and for the first mode the Davis-Kahan
    bound ||E||_2 / (lam_R - lam_{R+1} - ||E||_2) with E the Gram's error."""
    print(f"sthosvd {prec} dims={dims} eps={eps} order={order}", flush=True)
    order = order or list(range(len(dims)))
    x = to_dev(X, dims)
    t = tk.sthosvd(x, eps, mode_order=order, prec=prec, dims=dims)
    ref = orc.sthosvd(X.astype(np.float64), dims, eps, order)
    assert t.core_dtype == tk.F32
    xh = t.reconstruct(out_dtype=torch.float64)
    x64 = x.to(torch.float64)
    e = float(torch.linalg.vector_norm((x64 - xh).reshape(-1)) / torch.linalg.vector_norm(x64.reshape(-1)))
    angles = [_principal_sin(ref.factors[n], t.factor(n).cpu().numpy()) if t.ranks[n] == ref.ranks[n] else None
              for n in range(len(dims))]
    n0 = order[0]
    E = tk.gram(x, n0, prec=prec, dims=dims).cpu().numpy() - orc.gram(X.astype(np.float64), dims, n0)
    e2 = float(np.linalg.norm(E, 2))
    lam = ref.eigenvalues[n0]
    R0 = ref.ranks[n0]
    gap = (lam[R0 - 1] - lam[R0] - e2) if R0 < len(lam) else np.inf
    dk = e2 / gap if gap > 0 else np.inf
    print(f"  ranks gpu={t.ranks} oracle={ref.ranks} relerr={e:.4e} (eps {eps}) "
          f"sin-angles={[None if a is None else float('%.3g' % a) for a in angles]} "
          f"first-mode DK bound={dk:.3g} precision={t.gram_precision}", flush=True)
    return t, ref, e, angles, dk, e2


def accepted_ranks(lam, thr, E, slack):
    """Ranks that the truncation rule may select from a Gram S + E, given the
    exact eigenvalues `lam` of S (descending) and the error matrix E.

    By Lidskii's theorem (Ky Fan's principle for sums of eigenvalues), the sum
    of the k smallest eigenvalues of S + E differs from that of S by at most
    the sum of the k largest singular values of E.  So the computed tail at
    rank r lies within kf[J - r] of the exact tail[r] (plus `slack` for the
    FP64 eigensolver and summation rounding), and r is selectable iff
    tail[r] <= thr + kf[J - r] + slack (it may fit) and, for r > 1,
    tail[r - 1] > thr - kf[J - r + 1] - slack (r - 1 may not fit)."""
    lam = np.clip(np.asarray(lam, dtype=np.float64), 0.0, None)
    J = lam.size
    tail = np.concatenate([np.cumsum(lam[::-1])[::-1], [0.0]])
    sv = np.linalg.svd(E, compute_uv=False)
    kf = np.concatenate([[0.0], np.cumsum(sv)])  # kf[k] = sum of the k largest singular values
    ok = set()
    for r in range(1, J + 1):
        fits = tail[r] <= thr + kf[J - r] + slack
        minimal = r == 1 or tail[r - 1] > thr - kf[J - r + 1] - slack
        if fits and minimal:
            ok.add(r)
    return ok


def composed_rank_check(tk, orc, X, dims, eps, order, prec, t_ranks):
    """Run the reduced-form mode loop from the single-step C ABI calls
    (tucker_gram, tucker_eig_truncate, tucker_ttm: the kernels tucker_sthosvd
    runs, in its order: the product of a mode kept at full rank, other than
    the last, is left for the end, since it changes no later Gram), and check
    every mode's rank against the oracle's exact eigenvalues of the GPU's own
    partial core at that step, accepting exactly the ranks that a Gram within
    the measured error of the exact one may select (accepted_ranks).  Also
    checks the Gram error against the form's per-entry bound and that the
    composed loop reproduces tucker_sthosvd's ranks.  Returns the per-mode
    (rank, accepted set, ||E||_2 / trace)."""
    N = len(dims)
    y = to_dev(X, dims)
    cur = list(dims)
    thr = None
    out = []
    for n in order:
        S, nrm = tk.gram(y, n, prec=prec, dims=cur, with_norm=True)
        if thr is None:
            thr = (eps * eps / N) * float(nrm.item())
        Y64 = y.double().cpu().numpy().reshape(-1)
        Sref = orc.gram(Y64, cur, n)
        lam_ref, _ = orc.eig(Sref)
        E = S.cpu().numpy() - Sref
        tr = float(np.trace(Sref))
        d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref))) + 1e-300
        assert (np.abs(E) / d).max() <= BOUND[prec], (n, (np.abs(E) / d).max())
        lam, U, R, _ = tk.eig_truncate(S, thr)
        J = cur[n]
        ok = accepted_ranks(lam_ref, thr, E, 64 * J * np.finfo(float).eps * tr)
        assert R in ok, (n, R, sorted(ok))
        out.append((n, R, sorted(ok), float(np.linalg.norm(E, 2)) / max(tr, 1e-300)))
        if R == J and n != order[-1]:
            continue  # a full-rank mode's product runs after the last step
        y = tk.ttm(y, n, U.t(), dims=cur, out_dtype=torch.float32, fp32_products=True)
        cur[n] = R
    ranks = [0] * N
    for n, R, _, _ in out:
        ranks[n] = R
    assert ranks == list(t_ranks), (ranks, t_ranks)
    print(f"  composed per-mode (mode, rank, accepted, |E|_2/tr): {out}", flush=True)
    return out


SIM = [((40, 36, 32, 11, 6), [0, 1, 2, 3, 4]), ((40, 36, 32, 11, 6), [4, 3, 0, 1, 2])]


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4])
@pytest.mark.parametrize("shape,order", SIM)
def test_sthosvd_reduced_matches_oracle(tk, orc, prec, eps, shape, order):
    """FP32-MFMA and BF16X6 Grams on a combustion-shaped float32 tensor:
    relative error within 1.05 eps; every mode's rank accepted against the
    oracle's exact eigenvalues of the GPU's own partial core with that mode's
    measured Gram error (composed_rank_check); at eps >= 1e-3 also the FP64
    oracle's ranks exactly and a first-mode subspace within the Davis-Kahan
    bound of the Gram's measured error."""
    X, dims, _ = synthetic.combustion(shape, nbumps=16, seed=31)
    t, ref, e, angles, dk, e2 = _mixed_report(tk, orc, X, dims, eps, order, prec)
    assert e <= 1.05 * eps
    composed_rank_check(tk, orc, X, dims, eps, order, prec, t.ranks)
    if eps >= 1e-3:
        assert t.ranks == ref.ranks
        assert angles[order[0]] <= max(dk, 1e-6)


@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_sthosvd_bf16x3_error_target(tk, orc, eps):
    """BF16X3 meets the 1.05 eps target at eps >= 1e-3 on this tensor; its Gram
    under-estimates (the dropped b1 c1' term), so its ranks are never above the
    oracle's; every mode's rank is accepted by the per-mode check.  Below that
    the bias exceeds the budget (reported by the benchmark, not asserted)."""
    X, dims, _ = synthetic.combustion(SIM[0][0], nbumps=16, seed=31)
    t, ref, e, angles, dk, e2 = _mixed_report(tk, orc, X, dims, eps, SIM[0][1], "bf16x3")
    assert e <= 1.05 * eps
    assert all(r <= q for r, q in zip(t.ranks, ref.ranks))
    composed_rank_check(tk, orc, X, dims, eps, SIM[0][1], "bf16x3", t.ranks)


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_sthosvd_reduced_fourier(tk, orc, prec):
    """Fourier-field tensor (2 space, 33 variables, time) in mode order 3,2,0,1:
    1.05 eps and the per-mode rank check on every mode."""
    X, dims = synthetic.fourier_fields((96, 80, 33, 40), nmodes=64, seed=41)
    t, ref, e, angles, dk, e2 = _mixed_report(tk, orc, X, dims, 1e-4, [3, 2, 0, 1], prec)
    assert e <= 1.05e-4
    composed_rank_check(tk, orc, X, dims, 1e-4, [3, 2, 0, 1], prec, t.ranks)


def test_reconstruct_fp32_core(tk, orc):
    """FP32 core reconstructed to FP32 (FP32 products) and to FP64 (FP64
    products) against the oracle's Multi-TTM of the same core and factors."""
    X, dims, _ = synthetic.combustion((40, 36, 32, 11, 6), nbumps=16, seed=31)
    t = tk.sthosvd(to_dev(X, dims), 1e-3, prec="fp32", dims=dims)
    core = t.core.cpu().numpy().astype(np.float64).reshape(-1)
    Us = [t.factor(n).cpu().numpy() for n in range(5)]
    ref = orc.Tucker(core=core, factors=Us, ranks=list(t.ranks), dims=list(dims), eigenvalues=None,
                     discarded=None, norm2=t.norm2, order=list(range(5)))
    begin, end = [3, 5, 0, 2, 1], [33, 30, 32, 9, 6]
    Zref, zd = orc.reconstruct(ref, begin, end)
    Aref, _ = orc.reconstruct(orc.Tucker(core=np.abs(core), factors=[np.abs(U) for U in Us], ranks=ref.ranks,
                                         dims=ref.dims, eigenvalues=None, discarded=None, norm2=0.0,
                                         order=ref.order), begin, end)
    Z64 = t.reconstruct(begin, end, out_dtype=torch.float64).cpu().numpy().reshape(-1)
    assert np.all(np.abs(Z64 - Zref) <= 1e-12 * Aref + 1e-300)
    Z32 = t.reconstruct(begin, end, out_dtype=torch.float32).cpu().numpy().reshape(-1).astype(np.float64)
    R = max(t.ranks)
    assert np.all(np.abs(Z32 - Zref) <= 5 * (R + 4) * U32 * Aref + U32 * np.abs(Zref) + 1e-300)
