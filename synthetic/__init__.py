"""Seeded synthetic input generators shared by the tests and the benchmark.

This module holds no step of the compression method (no Gram, eigensolve,
truncation or TTM of the method's own); it only builds input tensors, with
numpy's PCG64 generator, following the synthetic-data recipe of the paper's
Sec. 9.2 (random core times random factors plus scaled Gaussian noise) as
adapted below.  It imports neither the oracle nor the GPU library.

Layout of every returned tensor: flat, natural descending (mode 0 fastest), so a
C-ordered array of shape ``dims[::-1]`` has the same bytes.

Adaptations of the paper's recipe (each stated where it is used):
* factors are orthonormal (QR of a Gaussian matrix, R's diagonal made positive)
  instead of Gaussian;
* the noise is scaled with its exact norm, so ||X - M|| / ||M|| equals eta
  exactly instead of approximately.
"""
from __future__ import annotations

import numpy as np


def _orthonormal(rng: np.random.Generator, I: int, R: int) -> np.ndarray:
    """I x R matrix with orthonormal columns: Q of a QR of an I x R Gaussian
    matrix, with the column signs chosen so that diag(R) > 0 (deterministic)."""
    Q, Rm = np.linalg.qr(rng.standard_normal((I, R)))
    s = np.sign(np.diag(Rm))
    s[s == 0] = 1.0
    return Q * s


def _expand(core: np.ndarray, core_dims, factors) -> np.ndarray:
    """Build core x_0 F_0 x_1 F_1 ... (input construction only), returning a
    flat natural-descending array.  ``core`` is flat natural-descending."""
    T = np.asarray(core, dtype=np.float64).reshape(tuple(core_dims[::-1]))  # axes: N-1 .. 0
    N = len(core_dims)
    for n, F in enumerate(factors):
        ax = N - 1 - n
        T = np.moveaxis(np.tensordot(F, T, axes=([1], [ax])), 0, ax)
    return np.ascontiguousarray(T).reshape(-1)


def _add_noise(rng: np.random.Generator, M: np.ndarray, eta: float) -> np.ndarray:
    """X = M + eta * (||M|| / ||E||) * E with E i.i.d. N(0,1) and the exact ||E||."""
    if eta == 0.0:
        return M
    E = rng.standard_normal(M.size)
    nm = np.sqrt(np.dot(M, M))
    ne = np.sqrt(np.dot(E, E))
    return M + (eta * nm / ne) * E


def random_tucker(dims, ranks, eta: float, seed: int, spectra=None, dtype=np.float64):
    """Random Tucker tensor plus noise.

    core ~ N(0,1)^{ranks}; if ``spectra`` is given (one ratio rho per mode) the
    core is scaled by diag(rho^r) along every mode r < R_n; factors orthonormal;
    X = M + eta ||M||/||E|| E.  Returns (X flat in ``dtype``, dims).
    """
    rng = np.random.default_rng(seed)
    dims = [int(v) for v in dims]
    ranks = [int(v) for v in ranks]
    core = rng.standard_normal(int(np.prod(ranks)))
    if spectra is not None:
        C = core.reshape(tuple(ranks[::-1]))
        N = len(ranks)
        for n, rho in enumerate(spectra):
            shape = [1] * N
            shape[N - 1 - n] = ranks[n]
            C = C * (float(rho) ** np.arange(ranks[n])).reshape(shape)
        core = np.ascontiguousarray(C).reshape(-1)
    factors = [_orthonormal(rng, I, R) for I, R in zip(dims, ranks)]
    M = _expand(core, ranks, factors)
    X = _add_noise(rng, M, eta)
    return X.astype(dtype), dims


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def lowrank_64():
    """64x64x64 float64: 8x8x8 N(0,1) core, orthonormal 64x8 factors, relative
    noise 1e-6 (seed 1).  Compressed with eps=1e-4, mode order 0,1,2."""
    return random_tucker([64, 64, 64], [8, 8, 8], 1e-6, seed=1)


def decaying_200(scale: int = 1):
    """200x200x200x16 float64 (``scale`` divides the three 200-sized modes for
    reduced test sizes): core 20x20x20x8 of N(0,1) entries scaled by 0.7^r along
    every mode, orthonormal factors, relative noise 1e-5 (seed 2)."""
    I = 200 // scale
    R = min(20, I)
    return random_tucker([I, I, I, 16], [R, R, R, 8], 1e-5, seed=2, spectra=[0.7] * 4)


def small_batch(count: int = 1024, lo: int = 16, hi: int = 128, base_seed: int = 4000,
                eta: float = 1e-4, dtype=np.float32):
    """``count`` independent 3-way tensors: sizes I_n ~ U{lo..hi}, ranks
    R_n ~ U{2..floor(I_n/4)}, Gaussian core, orthonormal factors, relative noise
    ``eta``; tensor i uses seed base_seed + i."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        dims = [int(v) for v in rng.integers(lo, hi + 1, size=3)]
        ranks = [int(rng.integers(2, max(2, d // 4) + 1)) for d in dims]
        X, _ = random_tucker(dims, ranks, eta, seed=base_seed + i + 1_000_000, dtype=dtype)
        out.append((X, dims))
    return out
