"""Parity of the FP64 path on the benchmark's large-share workload: the
672x672x33x626 float32 Fourier-field tensor (seed 5), eps = 1e-4, mode order
3,2,0,1, in the launch configuration bench.py times.

* Full size (37.3 GB): the oracle cannot compress it within a test, so
  - sampled entries of the first (mode-3) Gram are checked against the
    oracle's Gram of the sampled rows (rows of the mode-3 unfolding are
    contiguous slices of the tensor), within the FP64 summation bound;
  - the result is checked by properties that hold at any size: Corollary 1
    (the squared error equals the discarded energy), the eps bound,
    orthonormal factors, the eigen-residual of the mode-3 factor against the
    Gram, and ||X||^2 against the trace of that Gram.
* Reduced size (the same generator on a 96x80x33x72 grid): the oracle's ranks
  and relative error within 1e-10.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ORDER = [3, 2, 0, 1]
EPS = 1e-4


@pytest.fixture(scope="module")
def tk():
    import paper_1901_06043_amd as tk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tk.lib()
    return tk


def test_large_share_reduced_grid_matches_oracle(tk, orc):
    X, dims = synthetic.fourier_fields((96, 80, 33, 72), nmodes=128, seed=5)
    print(f"large share reduced dims={dims}", flush=True)
    x = torch.from_numpy(X.reshape(dims[::-1])).cuda()
    t = tk.sthosvd(x, EPS, mode_order=ORDER, prec="fp64")
    ref = orc.sthosvd(X.astype(np.float64), dims, EPS, ORDER)
    assert t.ranks == ref.ranks
    xh = t.reconstruct(out_dtype=torch.float64)
    x64 = x.double()
    e = float(torch.linalg.vector_norm((x64 - xh).reshape(-1)) / torch.linalg.vector_norm(x64.reshape(-1)))
    assert abs(e - orc.relerr(X.astype(np.float64), ref)) <= 1e-10
    assert e <= EPS


def test_large_share_full_size(tk, orc):
    print("large share full size: generating 672x672x33x626", flush=True)
    x, dims = synthetic.fourier_fields(device="cuda")
    assert dims == [672, 672, 33, 626]
    torch.cuda.synchronize()
    t = tk.sthosvd(x, EPS, mode_order=ORDER, prec="fp64")
    print(f"  ranks {t.ranks}", flush=True)
    # mode-3 Gram (the first step's kernel and plan) on sampled rows
    S = tk.gram(x, 3, dims=dims)
    J = dims[3]
    rows = [0, 1, 313, 624, 625]
    sub = x.view(J, -1)[rows].double().cpu().numpy()  # rows of the mode-3 unfolding
    L = sub.shape[1]
    Sref = orc.gram(sub.reshape(-1), [L, len(rows)], 1)
    d = np.sqrt(np.outer(np.diag(Sref), np.diag(Sref)))
    got = S.cpu().numpy()[np.ix_(rows, rows)]
    assert np.all(np.abs(got - Sref) <= 1e-11 * d), (np.abs(got - Sref) / d).max()
    # ||X||^2 (FP64, fused into the first Gram) equals trace S
    assert t.norm2 == pytest.approx(float(torch.trace(S)), rel=1e-12)
    # eigen-residual and orthonormality of the mode-3 factor
    U3 = t.factor(3)
    lam3 = t.eigenvalues(3)[: t.ranks[3]]
    res = torch.linalg.matrix_norm(S @ U3 - U3 * lam3, ord=2)
    assert float(res) <= 1e-11 * float(t.eigenvalues(3)[0])
    for n in range(4):
        U = t.factor(n)
        assert float((U.t() @ U - torch.eye(t.ranks[n], dtype=torch.float64, device="cuda")).abs().max()) <= 1e-12
    # Corollary 1 and the eps bound by explicit reconstruction, in slabs of time steps
    num = 0.0
    step = 63
    for s0 in range(0, dims[3], step):
        s1 = min(dims[3], s0 + step)
        xh = t.reconstruct([0, 0, 0, s0], [672, 672, 33, s1], out_dtype=torch.float64)
        num += float((x[s0:s1].double() - xh).pow(2).sum())
        del xh
    e2 = num / t.norm2
    assert np.sqrt(e2) <= EPS
    assert abs(e2 - sum(t.discarded) / t.norm2) <= 1e-11
    t.free()
    del x, S
    torch.cuda.empty_cache()
