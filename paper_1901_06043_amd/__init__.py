"""MI355X (gfx950) ST-HOSVD Tucker compression: thin Python binding.

Every computation runs in the HIP library ``libtuckerhip.so`` (built from
``csrc/`` by ``build.py``) through its C ABI (``include/tucker.h``).  This
module only marshals arguments: torch tensors provide device memory and the
current HIP stream.  There is no CPU fallback: if the library is missing or no
gfx950 device is present, calls raise.

Tensor convention: the paper's natural-descending layout (mode 0 fastest).  A
C-contiguous torch tensor of shape (I_{N-1}, ..., I_0) holds a tensor with
dims (I_0, ..., I_{N-1}); ``dims`` below are always in the paper's order.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtuckerhip.so")

F32, F64 = 0, 1
GRAM_FP64, GRAM_FP32, GRAM_BF16X3, GRAM_BF16X6, GRAM_AUTO = 0, 1, 2, 3, 4
_PREC = {"fp64": GRAM_FP64, "fp32": GRAM_FP32, "bf16x3": GRAM_BF16X3, "bf16x6": GRAM_BF16X6, "auto": GRAM_AUTO}
PREC_NAMES = {v: k for k, v in _PREC.items()}
PREC_CODES = dict(_PREC)
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EHIP", 4: "ENOCONV", 5: "EUNSUPPORTED"}
MAX_MODES = 16

EXPORTS = [
    "tucker_sthosvd", "tucker_ndims", "tucker_dims", "tucker_ranks", "tucker_mode_order", "tucker_core",
    "tucker_factor", "tucker_eigenvalues", "tucker_norm2", "tucker_discarded", "tucker_timings",
    "tucker_gram_precision", "tucker_free", "tucker_reconstruct", "tucker_reconstruct_order", "tucker_gram",
    "tucker_eig_truncate", "tucker_ttm", "tucker_last_error", "tucker_version",
    "tucker_batch_create", "tucker_batch_run", "tucker_sthosvd_batched", "tucker_batch_ranks",
    "tucker_batch_norm2", "tucker_batch_item", "tucker_batch_tiles", "tucker_batch_free",
    "tucker_op_size", "tucker_reconstruct_order_rule", "tucker_reconstruct_ops", "tucker_slice_stats",
    "tucker_scaling_vectors", "tucker_slice_transform", "tucker_preprocess", "tucker_set_postprocess",
    "tucker_create", "tucker_sthosvd_ranks", "tucker_sthosvd_memory", "tucker_set_allocator", "tucker_gram_scaled",
    "tucker_batch_status", "tucker_empty_cache", "tucker_eig_truncate_noalloc",
    "tucker_sthosvd_order",
]

OP_KINDS = {"identity": 0, "range": 1, "average": 2, "sum": 3, "mean": 4, "matrix": 5}
ORDER_RULES = {"flops": 0, "memory": 1}
SCALE_METHODS = {"standardize": 0, "max": 1}
STAT_NAMES = ["mean", "std", "min", "max", "norm1", "norm2"]


class _Op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("begin", ctypes.c_int64), ("end", ctypes.c_int64),
                ("step", ctypes.c_int64), ("rows", ctypes.c_int64), ("matrix", ctypes.c_void_p)]

_lib = None


class TuckerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


def lib():
    """Load libtuckerhip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1901_06043_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        PP = ctypes.POINTER(ctypes.c_void_p)
        sig = {
            "tucker_sthosvd": (i32, [P, i32, P, i32, d, P, i32, P, PP]),
            "tucker_ndims": (i32, [P]),
            "tucker_dims": (i32, [P, P]),
            "tucker_ranks": (i32, [P, P]),
            "tucker_mode_order": (i32, [P, P]),
            "tucker_core": (P, [P, P]),
            "tucker_factor": (P, [P, i32]),
            "tucker_eigenvalues": (P, [P, i32, P]),
            "tucker_norm2": (d, [P]),
            "tucker_discarded": (i32, [P, P]),
            "tucker_timings": (i32, [P, P]),
            "tucker_gram_precision": (i32, [P, P]),
            "tucker_free": (None, [P]),
            "tucker_reconstruct": (i32, [P, P, P, P, P, i32, P]),
            "tucker_reconstruct_order": (i32, [i32, P, P, P]),
            "tucker_gram": (i32, [P, i32, P, i32, i32, i32, P, P, P]),
            "tucker_eig_truncate": (i32, [P, i64, d, P, P, P, P, P]),
            "tucker_ttm": (i32, [P, i32, P, i32, i32, P, i64, i64, i64, P, i32, i32, P]),
            "tucker_batch_create": (i32, [i32, P, i32, P, i32, d, P, i32, P, PP]),
            "tucker_batch_run": (i32, [P, P]),
            "tucker_sthosvd_batched": (i32, [i32, P, i32, P, i32, d, P, i32, P, PP]),
            "tucker_batch_ranks": (i32, [P, P]),
            "tucker_batch_norm2": (i32, [P, P]),
            "tucker_batch_item": (i32, [P, i32, PP]),
            "tucker_batch_tiles": (i32, [P, P, P]),
            "tucker_batch_free": (None, [P]),
            "tucker_op_size": (i32, [P, i64, P]),
            "tucker_reconstruct_order_rule": (i32, [i32, P, P, i32, P]),
            "tucker_reconstruct_ops": (i32, [P, P, P, i32, P, i32, P]),
            "tucker_slice_stats": (i32, [P, i32, P, i32, i32, P, P]),
            "tucker_scaling_vectors": (i32, [P, i64, i32, P, P, P]),
            "tucker_slice_transform": (i32, [P, i32, P, i32, i32, P, P, i32, P, i32, P]),
            "tucker_preprocess": (i32, [P, i32, P, i32, i32, i32, P, i32, P, P, P]),
            "tucker_set_postprocess": (i32, [P, i32, P, P, P]),
            "tucker_create": (i32, [P, i32, P, P, i32, P, P, PP]),
            "tucker_sthosvd_ranks": (i32, [P, i32, P, i32, P, P, i32, P, PP]),
            "tucker_sthosvd_memory": (i32, [i32, P, i32, P, P, i32, P]),
            "tucker_set_allocator": (i32, [P]),
            "tucker_gram_scaled": (i32, [P, P]),
            "tucker_batch_status": (i32, [P, P]),
            "tucker_empty_cache": (i32, []),
            "tucker_sthosvd_order": (i32, [i32, P, P, P, P]),
            "tucker_eig_truncate_noalloc": (i32, [P, i64, d, P, P, P, P, P]),
            "tucker_last_error": (ctypes.c_char_p, []),
            "tucker_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise TuckerError(status, lib().tucker_last_error().decode(errors="replace"))


def _i64(vals):
    arr = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def _i32(vals):
    return (ctypes.c_int * len(vals))(*[int(v) for v in vals])


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _dims_of(x, dims):
    if dims is None:
        dims = list(reversed(x.shape))
    dims = [int(v) for v in dims]
    n = 1
    for v in dims:
        n *= v
    if x.numel() != n:
        raise ValueError(f"tensor has {x.numel()} elements, dims {dims} need {n}")
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if not x.is_cuda:
        raise ValueError("tensor must live on the GPU")
    return dims


class _DevArray:
    """Exposes handle-owned device memory to torch via __cuda_array_interface__."""

    def __init__(self, ptr: int, shape, typestr: str, owner):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}
        self._owner = owner


def _view(ptr, shape, typestr, owner):
    import torch
    return torch.as_tensor(_DevArray(ptr, shape, typestr, owner), device="cuda")


@dataclass
class Timing:
    gram_ms: float         # Gram step: main kernel + split-K reduction + norm
    eig_ms: float          # eigensolve + truncation
    ttm_ms: float
    gram_kernel_ms: float  # main Gram kernel alone


class Tucker:
    """Result of tucker_sthosvd: core, factors, ranks, eigenvalues (device memory
    owned by the C handle; tensors returned here are views kept alive by this
    object)."""

    def __init__(self, handle: int, stream: int, requested_precision: str = "fp64"):
        self._h = handle
        self._stream = stream
        self.requested_precision = requested_precision
        _live.add(self)
        L = lib()
        self.N = L.tucker_ndims(handle)
        d = (ctypes.c_int64 * self.N)()
        _check(L.tucker_dims(handle, d))
        self.dims = list(d)
        r = (ctypes.c_int64 * self.N)()
        _check(L.tucker_ranks(handle, r))
        self.ranks = list(r)
        o = (ctypes.c_int * self.N)()
        _check(L.tucker_mode_order(handle, o))
        self.mode_order = list(o)
        self.norm2 = float(L.tucker_norm2(handle))
        disc = (ctypes.c_double * self.N)()
        _check(L.tucker_discarded(handle, disc))
        self.discarded = list(disc)
        ms = (ctypes.c_double * (4 * self.N))()
        _check(L.tucker_timings(handle, ms))
        self.timings = [Timing(ms[4 * n], ms[4 * n + 1], ms[4 * n + 2], ms[4 * n + 3]) for n in range(self.N)]
        gp = (ctypes.c_int * self.N)()
        _check(L.tucker_gram_precision(handle, gp))
        # per mode: the Gram arithmetic used ("fp64" where the range handling fell back to it)
        self.gram_precision = [PREC_NAMES[v] for v in gp]
        sc = (ctypes.c_int * self.N)()
        _check(L.tucker_gram_scaled(handle, sc))
        # per mode: True if the Gram ran on the per-slice scaled copy
        self.gram_scaled = [bool(v) for v in sc]

    def _alive(self):
        if not self._h:
            raise RuntimeError("Tucker handle already freed")

    @property
    def core(self):
        """Core tensor G as a torch view of shape ranks[::-1] (natural descending)."""
        self._alive()
        dt = ctypes.c_int(0)
        p = lib().tucker_core(self._h, ctypes.byref(dt))
        return _view(p, list(reversed(self.ranks)), "<f8" if dt.value == F64 else "<f4", self)

    @property
    def core_dtype(self) -> int:
        dt = ctypes.c_int(0)
        lib().tucker_core(self._h, ctypes.byref(dt))
        return dt.value

    def factor(self, n: int):
        """U_n, I_n x R_n with orthonormal columns (a torch view)."""
        self._alive()
        p = lib().tucker_factor(self._h, n)
        # column-major I x R == C-ordered (R, I); return its transpose view
        return _view(p, (self.ranks[n], self.dims[n]), "<f8", self).t()

    @property
    def factors(self):
        return [self.factor(n) for n in range(self.N)]

    def eigenvalues(self, n: int):
        self._alive()
        cnt = ctypes.c_int64(0)
        p = lib().tucker_eigenvalues(self._h, n, ctypes.byref(cnt))
        return _view(p, (cnt.value,), "<f8", self)

    def reconstruct(self, begin=None, end=None, order=None, out_dtype=None, out=None, stream=None):
        """Sub-tensor X^[begin:end) by Multi-TTM (paper Sec. 8); returns a torch
        tensor of shape (end-begin)[::-1]."""
        import torch
        self._alive()
        b = list(begin) if begin is not None else [0] * self.N
        e = list(end) if end is not None else list(self.dims)
        shape = [int(e[k]) - int(b[k]) for k in range(self.N)]
        if out is None:
            if out_dtype is None:
                out_dtype = torch.float64 if self.core_dtype == F64 else torch.float32
            out = torch.empty(list(reversed(shape)), dtype=out_dtype, device="cuda")
        code = _dtype_code(out)
        _check(lib().tucker_reconstruct(self._h, _i64(b), _i64(e), _i32(order) if order is not None else None,
                                        out.data_ptr(), code, _stream(stream)))
        return out

    def reconstruct_ops(self, ops=None, order=None, rule="flops", out_dtype=None, out=None, stream=None):
        """Z = G x_n (C_n^T U_n) for per-mode operators (paper Sec. 8); ``ops`` is
        a list of N entries: None, ("range", b, e, step), ("average", b, e, w),
        ("sum", b, e), ("mean", b, e) or ("matrix", Ct) with Ct a K x I_n float64
        GPU tensor.  Returns a torch tensor of shape K[::-1]."""
        import torch
        self._alive()
        arr, keep = _ops_array(ops, self.N)
        K = [op_size(None if ops is None else ops[n], self.dims[n]) for n in range(self.N)]
        if out is None:
            if out_dtype is None:
                out_dtype = torch.float64 if self.core_dtype == F64 else torch.float32
            out = torch.empty(list(reversed(K)), dtype=out_dtype, device="cuda")
        _check(lib().tucker_reconstruct_ops(self._h, arr, _i32(order) if order is not None else None,
                                            ORDER_RULES[rule], out.data_ptr(), _dtype_code(out), _stream(stream)))
        del keep
        return out

    def set_postprocess(self, n: int, shift, scale, stream=None):
        """Attach the mode-n pre-processing vectors (paper Sec. 3.5) so that every
        reconstruction returns data in the original units; shift may be None."""
        self._alive()
        _check(lib().tucker_set_postprocess(self._h, int(n), None if shift is None else _f64_dev(shift).data_ptr(),
                                            _f64_dev(scale).data_ptr(), _stream(stream)))

    def free(self):
        if self._h:
            lib().tucker_free(self._h)
            self._h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _f64_dev(v):
    import torch
    if not (v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()):
        raise ValueError("expected a contiguous float64 GPU tensor")
    return v


def _ops_array(ops, N):
    """ctypes array of N tucker_op from the Python operator specs (and the
    tensors that must stay alive during the call)."""
    if ops is None:
        return None, []
    if len(ops) != N:
        raise ValueError(f"need {N} operators")
    arr = (_Op * N)()
    keep = []
    for n, op in enumerate(ops):
        if op is None:
            arr[n] = _Op(0, 0, 0, 1, 0, None)
            continue
        kind = op[0]
        if kind in ("range", "average"):
            arr[n] = _Op(OP_KINDS[kind], int(op[1]), int(op[2]), int(op[3]), 0, None)
        elif kind in ("sum", "mean"):
            arr[n] = _Op(OP_KINDS[kind], int(op[1]), int(op[2]), 1, 0, None)
        elif kind == "matrix":
            Ct = _f64_dev(op[1])
            keep.append(Ct)
            arr[n] = _Op(OP_KINDS[kind], 0, 0, 1, int(Ct.shape[0]), Ct.data_ptr())
        else:
            raise ValueError(f"unknown operator {kind}")
    return arr, keep


def op_size(op, I: int) -> int:
    """K of an operator spec on a mode of size I (host rule of the library)."""
    arr, keep = _ops_array([op], 1)
    if arr is None:
        return int(I)
    K = ctypes.c_int64(0)
    _check(lib().tucker_op_size(ctypes.byref(arr[0]), int(I), ctypes.byref(K)))
    return K.value


def reconstruct_order_rule(ranks, out_sizes, rule="flops"):
    N = len(ranks)
    o = (ctypes.c_int * N)()
    _check(lib().tucker_reconstruct_order_rule(N, _i64(ranks), _i64(out_sizes), ORDER_RULES[rule], o))
    return list(o)


def slice_stats(x, n: int, dims=None, stream=None):
    """Statistics of the hyperslices of mode n (paper Sec. 3.5): a (6, I_n) float64
    GPU tensor with rows mean, std, min, max, 1-norm, 2-norm."""
    import torch
    dims = _dims_of(x, dims)
    st = torch.empty((6, dims[n]), dtype=torch.float64, device=x.device)
    _check(lib().tucker_slice_stats(x.data_ptr(), _dtype_code(x), _i64(dims), len(dims), int(n), st.data_ptr(),
                                    _stream(stream)))
    return st


def scaling_vectors(stats, method: str, stream=None):
    """(shift, scale) of "standardize" or "max" from slice statistics."""
    import torch
    stats = _f64_dev(stats)
    J = stats.shape[1]
    shift = torch.empty(J, dtype=torch.float64, device=stats.device)
    scale = torch.empty(J, dtype=torch.float64, device=stats.device)
    _check(lib().tucker_scaling_vectors(stats.data_ptr(), J, SCALE_METHODS[method], shift.data_ptr(),
                                        scale.data_ptr(), _stream(stream)))
    return shift, scale


def slice_transform(x, n: int, shift, scale, inverse: bool = False, out=None, out_dtype=None, dims=None,
                    stream=None):
    """(x - shift_i) / scale_i along mode n (or the inverse x * scale_i + shift_i);
    ``out`` may be ``x`` (in place)."""
    import torch
    dims = _dims_of(x, dims)
    if out is None:
        out = torch.empty(x.shape, dtype=out_dtype or x.dtype, device=x.device)
    _check(lib().tucker_slice_transform(x.data_ptr(), _dtype_code(x), _i64(dims), len(dims), int(n),
                                        _f64_dev(shift).data_ptr(), _f64_dev(scale).data_ptr(), int(bool(inverse)),
                                        out.data_ptr(), _dtype_code(out), _stream(stream)))
    return out


def preprocess(x, n: int, method: str, out=None, dims=None, stream=None):
    """Statistics + vectors + forward map in one call: returns (y, shift, scale)."""
    import torch
    dims = _dims_of(x, dims)
    if out is None:
        out = torch.empty_like(x)
    shift = torch.empty(dims[n], dtype=torch.float64, device=x.device)
    scale = torch.empty(dims[n], dtype=torch.float64, device=x.device)
    _check(lib().tucker_preprocess(x.data_ptr(), _dtype_code(x), _i64(dims), len(dims), int(n),
                                   SCALE_METHODS[method], out.data_ptr(), _dtype_code(out), shift.data_ptr(),
                                   scale.data_ptr(), _stream(stream)))
    return out, shift, scale


def sthosvd(x, eps: float, mode_order=None, prec: str = "fp64", dims=None, stream=None) -> Tucker:
    """ST-HOSVD of a GPU tensor (paper Alg. 1) -> Tucker handle."""
    dims = _dims_of(x, dims)
    h = ctypes.c_void_p(0)
    s = _stream(stream)
    _check(lib().tucker_sthosvd(x.data_ptr(), _dtype_code(x), _i64(dims), len(dims), float(eps),
                                _i32(mode_order) if mode_order is not None else None, _PREC[prec], s,
                                ctypes.byref(h)))
    return Tucker(h.value, s, prec)


def from_model(core, factors, dims=None, stream=None) -> Tucker:
    """A handle from a given Tucker model: ``core`` a GPU tensor of shape
    ranks[::-1] (float32 or float64), ``factors`` the N float64 GPU matrices
    U_n (I_n x R_n, any strides; copied column-major)."""
    import torch
    N = len(factors)
    ranks = [int(U.shape[1]) for U in factors]
    dims = [int(U.shape[0]) for U in factors] if dims is None else list(dims)
    if not core.is_contiguous() or core.numel() != int(np.prod(ranks)):
        raise ValueError("core must be contiguous with prod(ranks) elements")
    cols = [U.to(torch.float64).t().contiguous() for U in factors]  # (R, I) C-order == I x R column-major
    ptrs = (ctypes.c_void_p * N)(*[c.data_ptr() for c in cols])
    h = ctypes.c_void_p(0)
    s = _stream(stream)
    _check(lib().tucker_create(core.data_ptr(), _dtype_code(core), _i64(dims), _i64(ranks), N, ptrs, s,
                               ctypes.byref(h)))
    return Tucker(h.value, s, "fp64")


def sthosvd_ranks(x, ranks, mode_order=None, prec: str = "fp64", dims=None, stream=None) -> Tucker:
    """Fixed-rank ST-HOSVD: R_n = min(ranks[n], J_n) (the core size is given)."""
    dims = _dims_of(x, dims)
    h = ctypes.c_void_p(0)
    s = _stream(stream)
    _check(lib().tucker_sthosvd_ranks(x.data_ptr(), _dtype_code(x), _i64(dims), len(dims), _i64(ranks),
                                      _i32(mode_order) if mode_order is not None else None, _PREC[prec], s,
                                      ctypes.byref(h)))
    return Tucker(h.value, s, prec)


def sthosvd_order(dims, ranks=None):
    """(mode order, predicted flops) by the Sec. 7 cost model; ranks None:
    increasing mode size."""
    N = len(dims)
    o = (ctypes.c_int * N)()
    f = ctypes.c_double(0.0)
    _check(lib().tucker_sthosvd_order(N, _i64(dims), _i64(ranks) if ranks is not None else None, o,
                                      ctypes.byref(f)))
    return list(o), f.value


def sthosvd_memory(dims, dtype: int = F64, ranks=None, mode_order=None, prec: str = "fp64") -> int:
    """Predicted device bytes of a compression (ranks None = no truncation bound)."""
    b = ctypes.c_size_t(0)
    _check(lib().tucker_sthosvd_memory(int(dtype), _i64(dims), len(dims), _i64(ranks) if ranks is not None else None,
                                       _i32(mode_order) if mode_order is not None else None, _PREC[prec],
                                       ctypes.byref(b)))
    return b.value


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)),
                ("ctx", ctypes.c_void_p)]


_torch_alloc = None
# bytes the library holds from PyTorch's allocator: live, peak since the last
# reset_allocator_stats(), and the number of alloc callbacks
allocator_stats = {"live": 0, "peak": 0, "calls": 0}
_torch_blocks = {}


def reset_allocator_stats():
    allocator_stats["peak"] = allocator_stats["live"]
    allocator_stats["calls"] = 0


def use_torch_allocator(enable: bool = True):
    """Route every device allocation of the library through PyTorch's caching
    allocator (tucker_set_allocator with ctypes callbacks), so that PyTorch
    provides the memory; enable=False restores the library's own pool (blocks
    taken from PyTorch go back to it when released)."""
    global _torch_alloc
    if not enable:
        _check(lib().tucker_set_allocator(None))
        return
    import torch

    def _alloc(nbytes, ctx, stream):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), stream or 0)
        except Exception:
            return None
        _torch_blocks[p] = int(nbytes)
        allocator_stats["live"] += int(nbytes)
        allocator_stats["peak"] = max(allocator_stats["peak"], allocator_stats["live"])
        allocator_stats["calls"] += 1
        return p

    def _free(ptr, ctx, stream):
        allocator_stats["live"] -= _torch_blocks.pop(ptr, 0)
        torch.cuda.caching_allocator_delete(ptr)

    a = _Allocator(_Allocator._fields_[0][1](_alloc), _Allocator._fields_[1][1](_free), None)
    _check(lib().tucker_set_allocator(ctypes.byref(a)))
    _torch_alloc = a  # the callbacks must outlive every block they produced


# Handles and plans still alive when the interpreter exits are released while
# Python still runs: their memory may belong to PyTorch's allocator, whose
# release goes through a Python callback.
_live = weakref.WeakSet()


@atexit.register
def _release_live():
    for obj in list(_live):
        try:
            obj.free()
        except Exception:
            pass


def empty_cache():
    """Return the library pool's idle device blocks to HIP."""
    _check(lib().tucker_empty_cache())


def reconstruct_order(ranks, out_sizes):
    """Flop-minimising Multi-TTM order (host rule of Sec. 8)."""
    N = len(ranks)
    o = (ctypes.c_int * N)()
    _check(lib().tucker_reconstruct_order(N, _i64(ranks), _i64(out_sizes), o))
    return list(o)


def gram(y, n: int, prec: str = "fp64", dims=None, with_norm: bool = False, stream=None):
    """S = Y_(n) Y_(n)^T (paper Alg. 2) as a J_n x J_n float64 tensor."""
    import torch
    dims = _dims_of(y, dims)
    J = dims[n]
    S = torch.empty((J, J), dtype=torch.float64, device=y.device)
    nrm = torch.empty((1,), dtype=torch.float64, device=y.device) if with_norm else None
    _check(lib().tucker_gram(y.data_ptr(), _dtype_code(y), _i64(dims), len(dims), n, _PREC[prec], S.data_ptr(),
                             nrm.data_ptr() if with_norm else None, _stream(stream)))
    return (S, nrm) if with_norm else S


def eig_truncate(S, thr: float, stream=None):
    """(lam descending, U leading columns, R, disc) of a symmetric J x J float64 matrix."""
    import torch
    J = S.shape[0]
    if S.dtype != torch.float64 or not S.is_contiguous() or tuple(S.shape) != (J, J):
        raise ValueError("S must be a contiguous J x J float64 tensor")
    lam = torch.empty((J,), dtype=torch.float64, device=S.device)
    Ubuf = torch.empty((J, J), dtype=torch.float64, device=S.device)
    R = torch.empty((1,), dtype=torch.int64, device=S.device)
    disc = torch.empty((1,), dtype=torch.float64, device=S.device)
    _check(lib().tucker_eig_truncate(S.data_ptr(), J, float(thr), lam.data_ptr(), Ubuf.data_ptr(), R.data_ptr(),
                                     disc.data_ptr(), _stream(stream)))
    r = int(R.item())
    # column-major J x J buffer: row k of Ubuf is column k of U
    return lam, Ubuf[:r].t(), r, float(disc.item())


def eig_truncate_noalloc(S, thr: float, lam, Ubuf, R, disc, stream=None):
    """tucker_eig_truncate_noalloc on caller-provided outputs (lam: J float64,
    Ubuf: J x J float64 whose row k receives eigenvector k, R: one int64,
    disc: one float64, all GPU tensors); the library allocates nothing."""
    J = S.shape[0]
    _check(lib().tucker_eig_truncate_noalloc(S.data_ptr(), J, float(thr), lam.data_ptr(), Ubuf.data_ptr(),
                                             R.data_ptr(), disc.data_ptr(), _stream(stream)))


def ttm(y, n: int, M, dims=None, out_dtype=None, fp32_products: bool = False, stream=None):
    """Z = Y x_n M (paper Sec. 2.2.3), M a K x J_n float64 tensor (any strides);
    fp32_products selects FP32 MFMA products instead of FP64."""
    import torch
    dims = _dims_of(y, dims)
    if M.dtype != torch.float64 or M.dim() != 2 or M.shape[1] != dims[n]:
        raise ValueError("M must be a K x J_n float64 matrix")
    K = M.shape[0]
    zd = list(dims)
    zd[n] = K
    if out_dtype is None:
        out_dtype = y.dtype
    Z = torch.empty(list(reversed(zd)), dtype=out_dtype, device=y.device)
    _check(lib().tucker_ttm(y.data_ptr(), _dtype_code(y), _i64(dims), len(dims), n, M.data_ptr(), K,
                            M.stride(0), M.stride(1), Z.data_ptr(), _dtype_code(Z), int(bool(fp32_products)),
                            _stream(stream)))
    return Z


class Batch:
    """Batched ST-HOSVD plan over many GPU tensors of the same order (every mode
    size <= 128): one run enqueues the whole compression (capturable in a HIP
    graph)."""

    def __init__(self, tensors, eps: float, mode_order=None, prec: str = "fp64", dims=None, stream=None):
        if len(tensors) == 0:
            raise ValueError("empty batch")
        dts = {_dtype_code(x) for x in tensors}
        if len(dts) != 1:
            raise ValueError("all tensors must have the same dtype")
        self.dims = [_dims_of(x, None if dims is None else dims[i]) for i, x in enumerate(tensors)]
        Ns = {len(dm) for dm in self.dims}
        if len(Ns) != 1:
            raise ValueError("all tensors must have the same order")
        self.N = Ns.pop()
        self.count = len(tensors)
        self._tensors = list(tensors)  # keep the inputs alive: the plan reads them at every run
        ptrs = (ctypes.c_void_p * self.count)(*[x.data_ptr() for x in tensors])
        flat = [v for dm in self.dims for v in dm]
        h = ctypes.c_void_p(0)
        _check(lib().tucker_batch_create(self.count, ptrs, dts.pop(), _i64(flat), self.N, float(eps),
                                         _i32(mode_order) if mode_order is not None else None, _PREC[prec],
                                         _stream(stream), ctypes.byref(h)))
        self._h = h.value
        _live.add(self)

    def run(self, stream=None):
        _check(lib().tucker_batch_run(self._h, _stream(stream)))

    def ranks(self):
        out = (ctypes.c_int64 * (self.count * self.N))()
        _check(lib().tucker_batch_ranks(self._h, out))
        return [list(out[i * self.N:(i + 1) * self.N]) for i in range(self.count)]

    def norm2(self):
        out = (ctypes.c_double * self.count)()
        _check(lib().tucker_batch_norm2(self._h, out))
        return list(out)

    def item(self, i: int) -> Tucker:
        h = ctypes.c_void_p(0)
        _check(lib().tucker_batch_item(self._h, int(i), ctypes.byref(h)))
        return Tucker(h.value, 0)

    def status(self):
        """Per tensor: 1 non-finite data, 2 a Gram recomputed in FP64 (bits)."""
        out = (ctypes.c_int * self.count)()
        _check(lib().tucker_batch_status(self._h, out))
        return list(out)

    def tiles(self):
        g, t = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib().tucker_batch_tiles(self._h, ctypes.byref(g), ctypes.byref(t)))
        return g.value, t.value

    def free(self):
        if self._h:
            lib().tucker_batch_free(self._h)
            self._h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

