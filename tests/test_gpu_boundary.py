"""GPU checks of the library's memory boundary and error reporting through
the C ABI: the device-memory prediction and ENOMEM before any launch, the
allocator hook (PyTorch's caching allocator provides the memory), and the
batched form's per-tensor range handling and status."""
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


def test_enomem_predicted_before_launch(tk):
    """With less free device memory than the first step needs (a filler
    allocation leaves half of the predicted amount), the call fails with
    ENOMEM from the prediction (its message names both figures) before any
    allocation; the data is a real tensor of the stated size throughout."""
    tk.empty_cache()
    torch.cuda.empty_cache()
    x = torch.randn((1000, 500, 500), dtype=torch.float32, device="cuda")  # dims 500 x 500 x 1000
    # what the first step needs (mode 0 untruncated, the later modes not yet known)
    need = tk.sthosvd_memory([500, 500, 1000], tk.F32, ranks=[500, 1, 1])
    assert need >= 500 * 500 * 1000 * 8
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    filler = torch.empty(free - need // 2, dtype=torch.uint8, device="cuda")
    try:
        with pytest.raises(tk.TuckerError) as ei:
            tk.sthosvd(x, 1e-2)
        assert ei.value.name == "ENOMEM"
        assert "available" in str(ei.value)
    finally:
        del filler
        torch.cuda.empty_cache()
    t = tk.sthosvd(x, 0.5)
    assert len(t.ranks) == 3
    t.free()
    del x
    torch.cuda.synchronize()


def test_allocator_hook_and_prediction_bound(tk, orc):
    """With PyTorch's caching allocator as the library's allocator, results are
    identical to the built-in pool's, every block comes through the callbacks
    (counted in the binding), the peak stays within the prediction for the
    actual ranks (which bounds every allocation of the run), and the blocks go
    back when the handle is freed."""
    X, dims = synthetic.random_tucker([120, 90, 60], [8, 7, 6], 1e-4, seed=3)
    x = to_dev(X, dims)
    ref = tk.sthosvd(x, 1e-3, dims=dims)
    core_ref = ref.core.clone()
    torch.cuda.synchronize()
    tk.use_torch_allocator(True)
    try:
        live0 = tk.allocator_stats["live"]
        tk.reset_allocator_stats()
        t = tk.sthosvd(x, 1e-3, dims=dims)
        peak = tk.allocator_stats["peak"] - live0
        held = tk.allocator_stats["live"] - live0
        assert tk.allocator_stats["calls"] > 0
        assert t.ranks == ref.ranks
        assert torch.equal(t.core, core_ref)
        assert held > 0  # the handle's core and factors live in PyTorch's pool
        pred = tk.sthosvd_memory(dims, tk.F64, ranks=t.ranks)
        assert 0 < peak <= pred, (peak, pred)
        xh = t.reconstruct()
        t.free()
        torch.cuda.synchronize()
        assert tk.allocator_stats["live"] == live0
        b = tk.Batch([x, x[:30].contiguous()], 1e-3, dims=[dims, [120, 90, 30]])
        b.run()
        assert b.ranks()[0] == ref.ranks
        b.free()
        assert tk.allocator_stats["live"] == live0
        del xh
    finally:
        tk.use_torch_allocator(False)
    torch.cuda.synchronize()


def test_batched_range_handling_and_status(tk, orc):
    """A batch mixing normal tensors with one whose values overflow FP32
    squares (1e20) and one holding a NaN: the overflowing tensor's Grams are
    recomputed in FP64 on the device (status bit 2) and get the oracle's
    ranks; the NaN tensor is reported (bit 0); the normal tensors are
    untouched (status 0, the same ranks as a batch without the others)."""
    data = synthetic.small_batch(count=6, base_seed=9100)
    X2 = (data[2][0].astype(np.float64) * 1e20).astype(np.float32)
    X4 = data[4][0].copy()
    X4[7] = np.nan
    xs = [to_dev(X, d, torch.float32) for X, d in data]
    xs[2] = to_dev(X2, data[2][1], torch.float32)
    xs[4] = to_dev(X4, data[4][1], torch.float32)
    dims = [d for _, d in data]
    b = tk.Batch(xs, 1e-2, prec="fp32", dims=dims)
    b.run()
    st = b.status()
    ranks = b.ranks()
    assert st[2] & 2 and not st[2] & 1
    assert st[4] & 1
    for i in (0, 1, 3, 5):
        assert st[i] == 0, (i, st)
    ref = orc.sthosvd(X2.astype(np.float64), dims[2], 1e-2)
    assert ranks[2] == ref.ranks
    clean = [xs[i] for i in (0, 1, 3, 5)]
    b2 = tk.Batch(clean, 1e-2, prec="fp32", dims=[dims[i] for i in (0, 1, 3, 5)])
    b2.run()
    assert b2.ranks() == [ranks[i] for i in (0, 1, 3, 5)]
    assert b2.status() == [0, 0, 0, 0]
    b.free()
    b2.free()
