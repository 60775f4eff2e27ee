"""The allocation-free eigensolver entry point (tucker_eig_truncate_noalloc,
static device workspace) against the allocating one (tucker_eig_truncate),
called through the C ABI: the same kernels on the same input, so the
eigenvalues, the rank, the discarded energy and the leading eigenvectors
must be bit-identical.  Calls run in a row with decreasing sizes (the largest
supported J first), so that each call finds the previous call's contents in
the shared workspace."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tk():
    import paper_1901_06043_amd as tk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tk.lib()
    return tk


def _outputs(J):
    f64 = dict(dtype=torch.float64, device="cuda")
    return (torch.full((J,), np.nan, **f64), torch.full((J, J), np.nan, **f64),
            torch.full((1,), -1, dtype=torch.int64, device="cuda"), torch.full((1,), np.nan, **f64))


def _gram(J, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((J, J + 7)) * (0.9 ** np.arange(J))[:, None]
    return A @ A.T


@pytest.mark.parametrize("sizes", [(1024, 300, 100), (209, 64, 1)])
def test_noalloc_matches_allocating_entry_point(tk, orc, sizes):
    L = tk.lib()
    stream = torch.cuda.current_stream().cuda_stream
    for k, J in enumerate(sizes):
        print(f"noalloc eig J={J}", flush=True)
        S = torch.from_numpy(_gram(J, 10 * J + k)).cuda()
        thr = 1e-6 * float(torch.trace(S))
        lam_a, U_a, R_a, d_a = _outputs(J)
        lam_b, U_b, R_b, d_b = _outputs(J)
        assert L.tucker_eig_truncate_noalloc(S.data_ptr(), J, thr, lam_a.data_ptr(), U_a.data_ptr(), R_a.data_ptr(),
                                             d_a.data_ptr(), stream) == 0
        assert L.tucker_eig_truncate(S.data_ptr(), J, thr, lam_b.data_ptr(), U_b.data_ptr(), R_b.data_ptr(),
                                     d_b.data_ptr(), stream) == 0
        torch.cuda.synchronize()
        R = int(R_a.item())
        assert R == int(R_b.item()) and 1 <= R <= J
        assert torch.equal(lam_a, lam_b)
        assert torch.equal(d_a, d_b)
        assert torch.equal(U_a[:R], U_b[:R])  # row k holds eigenvector k
        # and the result is the eigensolver's (the oracle's eigenvalues, orthonormal vectors)
        lref, _ = orc.eig(S.cpu().numpy())
        nS = float(np.abs(lref).max())
        assert np.abs(lam_a.cpu().numpy() - lref).max() <= 1e-12 * nS
        U = U_a[:R].cpu().numpy()
        assert np.abs(U @ U.T - np.eye(R)).max() <= 1e-12


def test_noalloc_rejects_sizes_beyond_its_workspace(tk):
    """J above the static workspace's 1024 is refused before any device work
    (the pointers are never read)."""
    L = tk.lib()
    dummy = ctypes.c_void_p(16)
    assert L.tucker_eig_truncate_noalloc(dummy, 1025, 0.0, dummy, dummy, dummy, dummy, None) == 1
    assert b"1024" in L.tucker_last_error()
    assert L.tucker_eig_truncate_noalloc(dummy, 0, 0.0, dummy, dummy, dummy, dummy, None) == 1
