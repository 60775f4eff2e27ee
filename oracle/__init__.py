"""FP64 CPU oracle for ST-HOSVD Tucker compression and Multi-TTM reconstruction.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library in ``paper_1901_06043_amd`` and never imports it.

The numeric kernels (Gram, Jacobi eigensolver, truncation, TTM) are plain C in
``oracle.c``; this module holds only the mode loop of the paper's Algorithm 1,
the reconstruction chain of Sec. 8 and an explicit error evaluator, written to
be read against the paper step by step.

Layout: a tensor is a flat float64 numpy array plus ``dims`` (mode 0 fastest,
paper Sec. 4.1).  A C-ordered numpy array of shape ``dims[::-1]`` has the same
bytes.  Factors are column-major ``I_n x R_n`` (stored as numpy arrays of shape
``(R_n, I_n)``, i.e. ``U.T`` in C order, exposed as ``(I_n, R_n)`` Fortran views).

Parity: every function here is pinned by ``tests/test_oracle_*.py`` against the
paper's printed worked example, closed-form identities (Theorem 1, Corollary 1,
the norm identity of Sec. 3), textbook special cases (Eckart-Young via an SVD)
and brute force on tiny inputs.  Absolute factor and core values on general
inputs have no printed value in the paper; they are pinned through those
identities, the SVD special case and brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _SO + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        P = ctypes.c_void_p
        lib.oracle_norm2.restype = d
        lib.oracle_norm2.argtypes = [P, i64]
        lib.oracle_unfold.restype = i32
        lib.oracle_unfold.argtypes = [P, P, i32, i32, P]
        lib.oracle_gram.restype = i32
        lib.oracle_gram.argtypes = [P, P, i32, i32, P, i32]
        lib.oracle_jacobi_eig.restype = i32
        lib.oracle_jacobi_eig.argtypes = [P, i32, P, P, i32]
        lib.oracle_truncate.restype = i32
        lib.oracle_truncate.argtypes = [P, i32, d, P]
        lib.oracle_sign_fix.restype = None
        lib.oracle_sign_fix.argtypes = [P, i64, i64]
        lib.oracle_ttm.restype = i32
        lib.oracle_ttm.argtypes = [P, P, i32, i32, P, i64, i64, i64, P, i32]
        lib.oracle_tail.restype = d
        lib.oracle_tail.argtypes = [P, i32, i32]
        lib.oracle_slice_stats.restype = i32
        lib.oracle_slice_stats.argtypes = [P, P, i32, i32, P]
        lib.oracle_slice_transform.restype = i32
        lib.oracle_slice_transform.argtypes = [P, P, i32, i32, P, P, i32, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _dims(dims) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int64))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


NTHREADS = 0  # 0 = OpenMP default (all cores of the affinity mask)


def norm2(x) -> float:
    x = _f64(x)
    return float(_load().oracle_norm2(_ptr(x), x.size))


def unfold(Y, dims, n: int) -> np.ndarray:
    """Mode-n unfolding as a dense J_n x (prod others) matrix (paper Sec. 2.2.1)."""
    Y = _f64(Y)
    d = _dims(dims)
    out = np.empty((int(d[n]), Y.size // int(d[n])), dtype=np.float64)
    if _load().oracle_unfold(_ptr(Y), _ptr(d), d.size, n, _ptr(out)) != 0:
        raise ValueError("bad shape")
    return out


def gram(Y, dims, n: int) -> np.ndarray:
    """S = Y_(n) Y_(n)^T (paper Alg. 2), J_n x J_n."""
    Y = _f64(Y)
    d = _dims(dims)
    J = int(d[n])
    S = np.empty((J, J), dtype=np.float64)
    if _load().oracle_gram(_ptr(Y), _ptr(d), d.size, n, _ptr(S), NTHREADS) != 0:
        raise ValueError("bad shape")
    return S


class NotConverged(RuntimeError):
    pass


def eig(S, max_sweeps: int = 60):
    """(lam descending, V column-major J x J as an (J, J) array with V[:, i] the i-th vector)."""
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float64))
    J = S.shape[0]
    lam = np.empty(J, dtype=np.float64)
    Vt = np.empty((J, J), dtype=np.float64)  # row i = eigenvector i (column-major V)
    sweeps = _load().oracle_jacobi_eig(_ptr(S), J, _ptr(lam), _ptr(Vt), max_sweeps)
    if sweeps < 0:
        raise NotConverged(f"Jacobi did not converge within {max_sweeps} sweeps")
    return lam, Vt.T


def truncate(lam, thr: float):
    lam = _f64(lam)
    disc = ctypes.c_double(0.0)
    R = _load().oracle_truncate(_ptr(lam), lam.size, float(thr), ctypes.byref(disc))
    return int(R), float(disc.value)


def sign_fix(U: np.ndarray) -> np.ndarray:
    """Return a copy of the I x R matrix U with each column's largest-|entry| positive."""
    Ut = np.ascontiguousarray(np.asarray(U, dtype=np.float64).T)  # column-major storage
    _load().oracle_sign_fix(_ptr(Ut), Ut.shape[1], Ut.shape[0])
    return Ut.T


def ttm(Y, dims, n: int, M) -> tuple[np.ndarray, list]:
    """Z = Y x_n M with M of shape (K, J_n) (paper Sec. 2.2.3, Alg. 3)."""
    Y = _f64(Y)
    d = _dims(dims)
    M = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
    K, J = M.shape
    if J != int(d[n]):
        raise ValueError("M has the wrong number of columns")
    zd = [int(v) for v in d]
    zd[n] = K
    Z = np.empty(int(np.prod(zd)), dtype=np.float64)
    rc = _load().oracle_ttm(_ptr(Y), _ptr(d), d.size, n, _ptr(M), K, J, 1, _ptr(Z), NTHREADS)
    if rc != 0:
        raise ValueError("bad shape")
    return Z, zd


@dataclass
class Tucker:
    core: np.ndarray            # flat, natural descending, sizes `ranks`
    factors: list               # U_n as (I_n, R_n) arrays
    ranks: list
    dims: list
    eigenvalues: list           # per mode, descending, length J_n (size of Y at that step)
    discarded: list             # per mode: sum of dropped eigenvalues (after clamping)
    norm2: float                # ||X||^2
    order: list = field(default_factory=list)


def tail(lam, R: int) -> float:
    """Energy discarded by keeping the R leading eigenvectors: the sum of the
    clamped eigenvalues lam[R:], accumulated from the smallest (Corollary 1)."""
    lam = _f64(lam)
    return float(_load().oracle_tail(_ptr(lam), lam.size, int(R)))


def sthosvd(X, dims, eps: float, order=None, max_sweeps: int = 60, ranks=None) -> Tucker:
    """ST-HOSVD of paper Alg. 1, step by step, in FP64.

    Y <- X; for each n in ``order``: S <- Y_(n) Y_(n)^T; (lam, V) <- eig(S)
    (descending); R_n <- smallest R whose discarded tail is <= eps^2 ||X||^2 / N
    (eq. Un); U_n <- V(:, 1:R_n) (sign convention: largest |entry| positive);
    Y <- Y x_n U_n^T.  Returns G = Y and the factors.

    ``ranks`` (the fixed-rank variant the paper mentions in Sec. 9.4.1: the
    user gives the core size and the error follows): R_n <- min(ranks[n], J_n)
    instead of the eq. Un rule; eps is then ignored.
    """
    dims = [int(v) for v in dims]
    N = len(dims)
    if N < 1 or any(v < 1 for v in dims):
        raise ValueError("dims must be positive")
    if ranks is None and (not (eps >= 0.0) or not np.isfinite(eps)):
        raise ValueError("eps must be finite and >= 0")
    if ranks is not None:
        ranks = [int(v) for v in ranks]
        if len(ranks) != N or any(v < 1 for v in ranks):
            raise ValueError("ranks must be N values >= 1")
    order = list(range(N)) if order is None else [int(v) for v in order]
    if sorted(order) != list(range(N)):
        raise ValueError("order must be a permutation of 0..N-1")
    Y = _f64(X)
    if Y.size != int(np.prod(dims)):
        raise ValueError("data size does not match dims")
    nx2 = norm2(Y)
    if not np.isfinite(nx2):
        raise ValueError("non-finite data")
    thr = eps * eps * nx2 / N if ranks is None else 0.0
    cur = list(dims)
    U = [None] * N
    R = [0] * N
    lams = [None] * N
    disc = [0.0] * N
    for n in order:
        S = gram(Y, cur, n)
        lam, V = eig(S, max_sweeps)
        if ranks is None:
            Rn, dn = truncate(lam, thr)
        else:
            Rn = min(ranks[n], cur[n])
            dn = tail(lam, Rn)
        Un = sign_fix(V[:, :Rn])
        Y, cur = ttm(Y, cur, n, Un.T)
        U[n], R[n], lams[n], disc[n] = Un, Rn, lam, dn
    return Tucker(core=Y, factors=U, ranks=R, dims=dims, eigenvalues=lams,
                  discarded=disc, norm2=nx2, order=order)


def reconstruct(t: Tucker, begin=None, end=None, order=None) -> tuple[np.ndarray, list]:
    """Sub-tensor of X^ = G x_0 U_0 ... x_{N-1} U_{N-1} (paper Sec. 8) over the
    half-open index ranges [begin_n, end_n): G x_n U_n[begin_n:end_n, :] for every
    n, applied one TTM at a time in ``order`` (any order gives the same result)."""
    N = len(t.dims)
    begin = [0] * N if begin is None else [int(v) for v in begin]
    end = list(t.dims) if end is None else [int(v) for v in end]
    order = list(range(N)) if order is None else [int(v) for v in order]
    Z, cur = _f64(t.core), list(t.ranks)
    for n in order:
        M = np.ascontiguousarray(t.factors[n][begin[n]:end[n], :])
        Z, cur = ttm(Z, cur, n, M)
    return Z, cur


def reconstruct_bruteforce(t: Tucker, begin=None, end=None) -> np.ndarray:
    """X^[i] = sum_r G[r] prod_n U_n[i_n, r_n] by explicit loops (tiny inputs only)."""
    N = len(t.dims)
    begin = [0] * N if begin is None else list(begin)
    end = list(t.dims) if end is None else list(end)
    out_dims = [e - b for b, e in zip(begin, end)]
    G = _f64(t.core)
    out = np.zeros(int(np.prod(out_dims)), dtype=np.float64)
    for lin_o in range(out.size):
        idx, rem = [], lin_o
        for n in range(N):
            idx.append(rem % out_dims[n] + begin[n])
            rem //= out_dims[n]
        s = 0.0
        for lin_g in range(G.size):
            rg, rem, p = [], lin_g, G[lin_g]
            for n in range(N):
                rn = rem % t.ranks[n]
                rem //= t.ranks[n]
                p *= t.factors[n][idx[n], rn]
            s += p
        out[lin_o] = s
    return out


def relerr(X, t: Tucker) -> float:
    """||X - X^|| / ||X|| by explicit full reconstruction, accumulated in FP64."""
    X = _f64(X)
    Xh, _ = reconstruct(t)
    nx = float(np.sqrt(norm2(X)))
    if nx == 0.0:
        return 0.0
    return float(np.sqrt(norm2(X - Xh)) / nx)


# ---------------------------------------------------------------------------
# Pre- and post-processing (paper Sec. 3.5)
# ---------------------------------------------------------------------------

STAT_NAMES = ["mean", "std", "min", "max", "norm1", "norm2"]


def slice_stats(Y, dims, n: int) -> np.ndarray:
    """Statistics of every hyperslice of mode n: a (6, J_n) array with rows
    mean, standard deviation (divided by the count), minimum, maximum, 1-norm
    and 2-norm (paper Sec. 3.5)."""
    Y = _f64(Y)
    d = _dims(dims)
    J = int(d[n])
    out = np.empty(6 * J, dtype=np.float64)
    if _load().oracle_slice_stats(_ptr(Y), _ptr(d), d.size, n, _ptr(out)) != 0:
        raise ValueError("bad shape")
    return out.reshape(6, J)


def scaling_vectors(stats: np.ndarray, method: str):
    """(shift, scale) of the two pre-processing methods of paper Sec. 3.5:
    "standardize" shifts by the mean and scales by the standard deviation;
    "max" scales by the largest absolute value (no shift).  A zero scale (a
    constant or all-zero slice) is replaced by 1, so the map stays invertible."""
    stats = np.asarray(stats, dtype=np.float64)
    if method == "standardize":
        shift = stats[0].copy()
        scale = stats[1].copy()
    elif method == "max":
        shift = np.zeros(stats.shape[1])
        scale = np.maximum(np.abs(stats[2]), np.abs(stats[3]))
    else:
        raise ValueError("method is 'standardize' or 'max'")
    scale[scale == 0.0] = 1.0
    return shift, scale


def slice_transform(Y, dims, n: int, shift, scale, inverse: bool = False) -> np.ndarray:
    """Per-hyperslice affine map along mode n: (Y - shift_i) / scale_i, or
    with ``inverse`` Y * scale_i + shift_i (one rounding)."""
    Y = _f64(Y)
    d = _dims(dims)
    sh, sc = _f64(shift), _f64(scale)
    if sh.size != int(d[n]) or sc.size != int(d[n]):
        raise ValueError("shift and scale need J_n values")
    Z = np.empty_like(Y)
    if _load().oracle_slice_transform(_ptr(Y), _ptr(d), d.size, n, _ptr(sh), _ptr(sc), int(bool(inverse)),
                                      _ptr(Z)) != 0:
        raise ValueError("bad shape")
    return Z


# ---------------------------------------------------------------------------
# Reconstruction through per-mode linear operators (paper Sec. 8)
# ---------------------------------------------------------------------------

def operator_matrix(op, I: int) -> np.ndarray:
    """The K x I matrix C^T of one mode's operator (paper Sec. 8: the mode-n
    factor U_n is replaced by C_n^T U_n).  ``op`` is None (identity) or a
    tuple:
      ("range", begin, end, step)   rows begin, begin+step, ... below end;
      ("average", begin, end, w)    row k = the mean of rows [begin+k*w,
                                    min(begin+(k+1)*w, end)) (down-sampling by
                                    averaging; the paper's example takes w=2);
      ("sum", begin, end)           one row: the sum of rows [begin, end);
      ("mean", begin, end)          one row: their mean;
      ("matrix", Ct)                a given K x I matrix.
    """
    if op is None:
        return np.eye(I)
    kind = op[0]
    if kind == "matrix":
        Ct = np.asarray(op[1], dtype=np.float64)
        if Ct.ndim != 2 or Ct.shape[1] != I:
            raise ValueError("matrix operator must be K x I")
        return Ct
    b, e = int(op[1]), int(op[2])
    if not (0 <= b < e <= I):
        raise ValueError("bad range")
    if kind == "range":
        step = int(op[3])
        rows = list(range(b, e, step))
        Ct = np.zeros((len(rows), I))
        for k, i in enumerate(rows):
            Ct[k, i] = 1.0
        return Ct
    if kind == "average":
        w = int(op[3])
        K = -(-(e - b) // w)
        Ct = np.zeros((K, I))
        for k in range(K):
            lo, hi = b + k * w, min(b + (k + 1) * w, e)
            Ct[k, lo:hi] = 1.0 / (hi - lo)
        return Ct
    if kind in ("sum", "mean"):
        Ct = np.zeros((1, I))
        Ct[0, b:e] = 1.0 if kind == "sum" else 1.0 / (e - b)
        return Ct
    raise ValueError(f"unknown operator {kind}")


def reconstruct_ops(t: Tucker, ops=None, order=None, post=None):
    """Z = X^ x_0 C_0^T x_1 ... x_{N-1} C_{N-1}^T (paper Sec. 8), written out
    plainly: the full reconstruction X^ = G x_n U_n (one TTM per mode in
    ``order``), then, if ``post`` = (m, shift, scale) is given, the inverse of
    the mode-m pre-processing X^ <- X^ * scale + shift (paper Sec. 3.5), then
    the operators as mode products in increasing mode order.  (Any order of
    the mode products gives the same result, up to rounding.)"""
    N = len(t.dims)
    ops = [None] * N if ops is None else list(ops)
    Xh, cur = reconstruct(t, order=order)
    if post is not None:
        m, shift, scale = post
        Xh = slice_transform(Xh, cur, m, shift, scale, inverse=True)
    Z = Xh
    for n in range(N):
        if ops[n] is None:
            continue
        Ct = operator_matrix(ops[n], t.dims[n])
        Z, cur = ttm(Z, cur, n, Ct)
    return Z, cur
