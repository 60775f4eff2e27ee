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


# ---------------------------------------------------------------------------
# Simulation-shaped float32 workloads (reduced-precision form)
# ---------------------------------------------------------------------------

def _bump_params(rng: np.random.Generator, nvar: int, nbumps: int):
    """Per variable v and bump b: centre ~ U[0,1)^3, width ~ U[0.03, 0.15],
    amplitude ~ N(0,1), velocity ~ U[-0.3, 0.3]^3 per unit time; per-variable
    scale 10^U[-6, 3]."""
    centre = rng.uniform(0.0, 1.0, size=(nvar, nbumps, 3))
    width = rng.uniform(0.03, 0.15, size=(nvar, nbumps))
    amp = rng.standard_normal((nvar, nbumps))
    vel = rng.uniform(-0.3, 0.3, size=(nvar, nbumps, 3))
    scale = 10.0 ** rng.uniform(-6.0, 3.0, size=nvar)
    return centre, width, amp, vel, scale


def combustion(dims=(256, 256, 256, 11, 50), nbumps: int = 64, seed: int = 3, device=None):
    """Combustion-shaped 5-way float32 tensor (3 space, variables, time steps).

    Variable v at time step s (t = s / T) is s_v * sum_b a_vb g_x g_y g_z, a sum of
    ``nbumps`` Gaussian bumps exp(-d^2 / (2 w_vb^2)) on the periodic unit cube
    (grid p_i = i / I, minimum-image distance d to the centre c_vb + u_vb t, one
    factor per axis), so each (v, t) slice is a sum of ``nbumps`` rank-1 terms;
    s_v = 10^U[-6, 3].  Every variable is then max-rescaled over space and time
    (its largest |value| becomes 1); the combined scale vector is returned.

    Returns (X, dims, scales): with ``device=None`` X is a flat numpy float32
    array computed in float64; otherwise a torch float32 tensor of shape
    dims[::-1] on ``device``, evaluated there in float32 from the same
    float64 profiles.
    """
    nx, ny, nz, nvar, nt = [int(v) for v in dims]
    rng = np.random.default_rng(seed)
    centre, width, amp, vel, scale = _bump_params(rng, nvar, nbumps)
    tt = np.arange(nt) / nt
    grids = [np.arange(n) / n for n in (nx, ny, nz)]

    def profiles(v, axis):
        # (nt, nbumps, n): exp(-d^2 / (2 w^2)), d the periodic distance to c + u t
        c = centre[v, :, axis][None, :] + vel[v, :, axis][None, :] * tt[:, None]
        d = grids[axis][None, None, :] - c[:, :, None]
        d -= np.round(d)
        return np.exp(-(d ** 2) / (2.0 * width[v][None, :, None] ** 2))

    maxes = np.zeros(nvar)
    if device is None:
        X = np.empty((nt, nvar, nz, ny, nx), dtype=np.float32)
        for v in range(nvar):
            gx, gy, gz = profiles(v, 0), profiles(v, 1), profiles(v, 2)
            blk = scale[v] * np.einsum("b,tbz,tby,tbx->tzyx", amp[v], gz, gy, gx, optimize=True)
            maxes[v] = np.abs(blk).max()
            X[:, v] = (blk / maxes[v]).astype(np.float32)
        return X.reshape(-1), [nx, ny, nz, nvar, nt], scale / maxes

    import torch
    X = torch.empty((nt, nvar, nz, ny, nx), dtype=torch.float32, device=device)
    for v in range(nvar):
        gx = torch.from_numpy(profiles(v, 0)).to(device, torch.float32)            # (nt, b, nx)
        gy = torch.from_numpy(profiles(v, 1)).to(device, torch.float32)            # (nt, b, ny)
        gz = torch.from_numpy(profiles(v, 2) * (scale[v] * amp[v])[None, :, None]).to(device, torch.float32)
        for t in range(nt):
            A = (gz[t][:, :, None] * gy[t][:, None, :]).reshape(nbumps, nz * ny)  # (b, nz*ny)
            X[t, v].view(nz * ny, nx).copy_(torch.mm(A.t().contiguous(), gx[t]))
        m = float(X[:, v].abs().max())
        maxes[v] = m
        X[:, v].div_(m)
    return X, [nx, ny, nz, nvar, nt], scale / maxes


def fourier_fields(dims=(672, 672, 33, 626), nmodes: int = 512, eta: float = 1e-4, seed: int = 5, device=None):
    """4-way float32 tensor (2 space, variables, time steps) of smooth random
    Fourier fields plus noise.

    Variable v at time step s (t = s / T) is sum_m A cos(2 pi (kx x + ky y) +
    2 pi w t + phi) over ``nmodes`` modes of its own, on the periodic grid
    x_i = i / I: (kx, ky) is the integer rounding of |k| (cos a, sin a) with
    |k| ~ U[1, 64] and a ~ U[0, 2 pi); A = xi |k|^(-5/6) with xi ~ N(0,1) (energy
    spectrum ~ |k|^(-5/3)); w ~ U[0, 8] cycles per window; phi ~ U[0, 2 pi).
    Each (v, t) slice is evaluated separably: cos(a + b + c) expands into
    products of cosines and sines of the x, y and t phases.  Gaussian noise is
    added with relative Frobenius norm ``eta`` (exact norm).

    Returns (X, dims): numpy flat float32 (computed in float64) with
    ``device=None``, else a torch float32 tensor of shape dims[::-1] on
    ``device`` (phases in float64 there, the separable products in float32,
    noise drawn with torch's generator).
    """
    nx, ny, nvar, nt = [int(v) for v in dims]
    rng = np.random.default_rng(seed)
    kmag = rng.uniform(1.0, 64.0, size=(nvar, nmodes))
    ang = rng.uniform(0.0, 2 * np.pi, size=(nvar, nmodes))
    kx = np.rint(kmag * np.cos(ang))
    ky = np.rint(kmag * np.sin(ang))
    A = rng.standard_normal((nvar, nmodes)) * kmag ** (-5.0 / 6.0)
    w = rng.uniform(0.0, 8.0, size=(nvar, nmodes))
    phi = rng.uniform(0.0, 2 * np.pi, size=(nvar, nmodes))
    tt = np.arange(nt) / nt

    def lhs(v):
        ax = 2 * np.pi * np.outer(np.arange(nx) / nx, kx[v])  # (nx, M)
        return np.concatenate([np.cos(ax), np.sin(ax)], axis=1)  # (nx, 2M)

    def rhs(v, ts):
        # (len(ts), ny, 2M) with field^T (ny x nx) = rhs @ lhs^T:
        # cos(a + b + c) = cos a [cos b cos c - sin b sin c] - sin a [sin b cos c + cos b sin c]
        ay = 2 * np.pi * np.outer(np.arange(ny) / ny, ky[v])   # (ny, M)
        Cy, Sy = np.cos(ay), np.sin(ay)
        psi = 2 * np.pi * w[v][None, :] * tt[ts][:, None] + phi[v][None, :]
        Dc, Ds = A[v] * np.cos(psi), A[v] * np.sin(psi)        # (nt', M)
        top = Cy[None] * Dc[:, None, :] - Sy[None] * Ds[:, None, :]
        bot = -Sy[None] * Dc[:, None, :] - Cy[None] * Ds[:, None, :]
        return np.concatenate([top, bot], axis=2)

    if device is None:
        X = np.empty((nt, nvar, ny, nx), dtype=np.float64)
        for v in range(nvar):
            X[:, v] = rhs(v, np.arange(nt)) @ lhs(v).T
        X = _add_noise(rng, X.reshape(-1), eta)
        return X.astype(np.float32), [nx, ny, nvar, nt]

    import torch
    X = torch.empty((nt, nvar, ny, nx), dtype=torch.float32, device=device)
    f64 = dict(dtype=torch.float64, device=device)
    xs = torch.arange(nx, **f64) / nx
    ys = torch.arange(ny, **f64) / ny
    tts = torch.from_numpy(tt).to(**f64)
    tb = 32
    for v in range(nvar):
        ax = 2 * np.pi * xs[:, None] * torch.from_numpy(kx[v]).to(**f64)[None, :]
        Pt = torch.cat([torch.cos(ax), torch.sin(ax)], dim=1).t().contiguous().float()  # (2M, nx)
        ay = 2 * np.pi * ys[:, None] * torch.from_numpy(ky[v]).to(**f64)[None, :]
        Cy, Sy = torch.cos(ay), torch.sin(ay)                                            # (ny, M)
        Av = torch.from_numpy(A[v]).to(**f64)
        wv = torch.from_numpy(w[v]).to(**f64)
        pv = torch.from_numpy(phi[v]).to(**f64)
        for t0 in range(0, nt, tb):
            t1 = min(nt, t0 + tb)
            psi = 2 * np.pi * wv[None, :] * tts[t0:t1, None] + pv[None, :]
            Dc, Ds = Av * torch.cos(psi), Av * torch.sin(psi)                             # (b, M)
            top = Cy[None] * Dc[:, None, :] - Sy[None] * Ds[:, None, :]
            bot = -Sy[None] * Dc[:, None, :] - Cy[None] * Ds[:, None, :]
            R = torch.cat([top, bot], dim=2).float()                                      # (b, ny, 2M)
            X[t0:t1, v] = torch.matmul(R, Pt)
    if eta > 0:
        # noise with exact relative norm eta, drawn on the device one time step at a time
        flat = X.view(nt, -1)
        nm2 = sum(float(flat[t].double().pow(2).sum()) for t in range(nt))
        g = torch.Generator(device=device)
        E = torch.empty_like(flat[0])
        g.manual_seed(seed)
        ne2 = 0.0
        for t in range(nt):
            E.normal_(generator=g)
            ne2 += float(E.double().pow(2).sum())
        c = eta * np.sqrt(nm2 / ne2)
        g.manual_seed(seed)
        for t in range(nt):
            E.normal_(generator=g)
            flat[t].add_(E, alpha=c)
    return X, [nx, ny, nvar, nt]
