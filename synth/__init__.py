"""Seeded synthetic snapshot matrices.

This module only manufactures inputs.  It contains none of the compressor's
arithmetic (no sketching, no pivoted QR, no interpolation coefficients), so both
the HIP product path and the CPU oracle can take their inputs from it.

The paper's data (DNS channel-flow fields and particle trajectories, Sec. 3)
are not available; the generators below stand in for them with the shapes and
structure the paper describes:

* ``spectral_snapshots`` -- channel-like velocity snapshots: a sum of random
  Fourier modes with a k^-5/3 energy spectrum, wall-damped profiles in y on a
  wall-clustered grid, and slowly drifting phases in time.  Rows are
  (component, x, y, z) grid points, z fastest; columns are snapshots.  The grid
  defaults follow the paper's DNS box (Sec. 3: 4*pi x 2 x 4*pi/3, stretched
  toward the walls in y).
* ``lowrank_exact_spectrum`` -- A = U diag(sigma) V^T (+ optional absolute
  noise) with U, V orthonormal from QR of seeded Gaussians.
* ``dct_lowrank`` -- A = U diag(sigma) V^T with U made of randomly signed,
  row-permuted orthonormal DCT-II columns, cheap to build at millions of rows.

Everything is generated with torch (CPU or GPU), in FP64, and returned as a
column-major matrix: a tensor of shape (n, N) whose transpose view is the
N x n matrix, so that ``t.T`` is A and every snapshot (column of A) is
contiguous.  ``as_colmajor``/``colmajor_view`` convert.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch


def colmajor_empty(N: int, n: int, dtype=torch.float32, device="cpu") -> torch.Tensor:
    """Storage for an N x n column-major matrix; returns the N x n view."""
    return torch.empty((n, N), dtype=dtype, device=device).T


def as_colmajor(A: torch.Tensor) -> torch.Tensor:
    """Copy A (N x n) into column-major storage and return the N x n view."""
    out = colmajor_empty(A.shape[0], A.shape[1], A.dtype, A.device)
    out.copy_(A)
    return out


@dataclass(frozen=True)
class SpectralConfig:
    nx: int = 128
    ny: int = 64
    nz: int = 64
    n_snapshots: int = 500
    n_modes: int = 400
    seed: int = 1001
    drift: float = 0.0385        # U_c: phase drift rate (radians per snapshot per unit wavenumber);
                                 # 0.0385 puts the k=100 ID error of the 128x64x64 x 500 field at 1.8e-3
    decorrelation: float = 0.1   # relative random drift per mode
    lx: float = 4.0 * math.pi
    lz: float = 4.0 * math.pi / 3.0
    kmax: float = 0.0            # largest wavelength count of a mode per extent (0: nz / 4);
                                 # small values give fields resolved on coarse grids

    @property
    def rows(self) -> int:
        return 3 * self.nx * self.ny * self.nz


def _modes(cfg: SpectralConfig):
    rng = np.random.default_rng(cfg.seed)
    q = cfg.n_modes
    mmax = cfg.kmax if cfg.kmax > 0.0 else max(cfg.nz / 4.0, 1.5)
    m = rng.uniform(1.0, mmax, size=q)                       # |kappa| in domain units
    d = rng.normal(size=(q, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)            # direction on the sphere
    e = rng.normal(size=(q, 3))
    e -= (e * d).sum(1, keepdims=True) * d                   # component direction, perpendicular
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    amp = m ** (-5.0 / 6.0)                                  # E(k) ~ k^-5/3 with uniform |k|
    phase0 = rng.uniform(0.0, 2.0 * math.pi, size=q)
    xi = rng.normal(size=q)
    # physical wavenumbers: m wavelengths across each (periodic-looking) extent
    kx = 2.0 * math.pi * m * d[:, 0] / cfg.lx
    ky = 2.0 * math.pi * m * d[:, 1] / 2.0
    kz = 2.0 * math.pi * m * d[:, 2] / cfg.lz
    omega = cfg.drift * m * (d[:, 0] + cfg.decorrelation * xi)  # radians per snapshot
    return dict(kx=kx, ky=ky, kz=kz, e=e, amp=amp, phase0=phase0, omega=omega)


def spectral_snapshots(cfg: SpectralConfig, dtype=torch.float32, device="cpu",
                       col0: int = 0, ncols: int | None = None,
                       rms: float | None = None) -> torch.Tensor:
    """Channel-like snapshot matrix (rows = grid points x components, columns =
    snapshots col0 .. col0+ncols-1), column-major N x ncols view.

    Each entry is sum_q a_q e_{q,c} f_c(y) cos(kappa_q . x + phi_q(t)) with
    phi_q(t) = phi_q0 + omega_q t, evaluated in FP64 as a product of a spatial
    factor (N x 2Q) and a temporal factor (2Q x ncols), rounded to dtype, then
    divided by ``rms`` (default: the RMS of the generated block itself, so a
    full matrix has unit RMS; pass the full matrix's value to make column
    blocks of one matrix share one scale -- see ``spectral_rms``).
    """
    if ncols is None:
        ncols = cfg.n_snapshots - col0
    md = _modes(cfg)
    dev = torch.device(device)
    f64 = torch.float64
    kx = torch.tensor(md["kx"], dtype=f64, device=dev)
    ky = torch.tensor(md["ky"], dtype=f64, device=dev)
    kz = torch.tensor(md["kz"], dtype=f64, device=dev)
    e = torch.tensor(md["e"], dtype=f64, device=dev)
    amp = torch.tensor(md["amp"], dtype=f64, device=dev)
    ph0 = torch.tensor(md["phase0"], dtype=f64, device=dev)
    om = torch.tensor(md["omega"], dtype=f64, device=dev)

    x = torch.arange(cfg.nx, dtype=f64, device=dev) * (cfg.lx / cfg.nx)
    z = torch.arange(cfg.nz, dtype=f64, device=dev) * (cfg.lz / cfg.nz)
    jj = torch.arange(cfg.ny, dtype=f64, device=dev)
    y = -torch.cos(math.pi * jj / max(cfg.ny - 1, 1))
    wall = 1.0 - y * y
    prof = [wall, wall * wall, wall]                          # u, v, w damping

    def cexp(coord, k):
        ang = coord[:, None] * k[None, :]
        return torch.complex(torch.cos(ang), torch.sin(ang))

    ex, ey, ez = cexp(x, kx), cexp(y, ky), cexp(z, kz)

    t = torch.arange(col0, col0 + ncols, dtype=f64, device=dev)
    phase = ph0[None, :] + t[:, None] * om[None, :]           # ncols x Q
    temporal = torch.cat([torch.cos(phase), -torch.sin(phase)], dim=1)

    N = cfg.rows
    out = torch.empty((ncols, N), dtype=dtype, device=dev)    # column-major storage
    plane = cfg.ny * cfg.nz
    sumsq = torch.zeros((), dtype=f64, device=dev)
    for c in range(3):
        wc = amp * e[:, c]                                     # Q
        pc = prof[c].repeat_interleave(cfg.nz)[:, None] * wc[None, :]
        eyz = (ey[:, None, :] * ez[None, :, :]).reshape(plane, -1)
        for i in range(cfg.nx):
            sp = (eyz * ex[i][None, :]) * pc                   # plane x Q complex
            F = torch.cat([sp.real, sp.imag], dim=1)           # plane x 2Q
            blk = temporal @ F.T                               # ncols x plane
            sumsq += torch.sum(blk * blk)
            r0 = (c * cfg.nx + i) * plane
            out[:, r0:r0 + plane] = blk.to(dtype)
    if rms is None:
        rms = float(torch.sqrt(sumsq / (N * ncols)))
    out /= rms
    return out.T


def streaming_config() -> SpectralConfig:
    """The streamed field: 1,572,864 x 2000 snapshots on the 128 x 64 x 64
    grid, sampled four times as densely in time as the 500-snapshot field
    relative to its decorrelation (drift 0.0155 rad per snapshot and unit
    wavenumber).  With the 500-snapshot field's drift the 2000 snapshots
    decorrelate completely (optimal rank-150 error 0.2); here the optimal
    rank-150 error is 2.6e-4 (from the exact Gram matrix of the spatial and
    temporal factors), so a rank-150 ID of it sits in the same regime as the
    rank-100 ID of the 500-snapshot field (optimal 3.2e-4)."""
    return SpectralConfig(n_snapshots=2000, drift=0.0155)


def spectral_rms(cfg: SpectralConfig) -> float:
    """RMS of the full (all snapshots) FP64 field, for scaling column blocks."""
    md = _modes(cfg)
    # sum over rows and columns of (F T)^2 computed plane by plane on a
    # coarse-in-time subsample would be approximate; generate exactly instead.
    A = spectral_snapshots(cfg, dtype=torch.float64, rms=1.0)
    return float(torch.sqrt(torch.mean(A.T.reshape(-1) ** 2)))


def lowrank_exact_spectrum(N: int, n: int, sigma: np.ndarray, seed: int,
                           noise: float = 0.0, dtype=torch.float64,
                           device="cpu") -> torch.Tensor:
    """A = U diag(sigma) V^T + noise * G (column-major N x n view).

    U (N x r) and V (n x r), r = len(sigma), are the Q factors of seeded
    Gaussian matrices (numpy PCG64 streams derived from ``seed``); G is an
    independent standard Gaussian N x n matrix.
    """
    r = len(sigma)
    rng_u = np.random.default_rng([seed, 1])
    rng_v = np.random.default_rng([seed, 2])
    U, _ = np.linalg.qr(rng_u.standard_normal((N, r)))
    V, _ = np.linalg.qr(rng_v.standard_normal((n, r)))
    A = (U * np.asarray(sigma, dtype=np.float64)[None, :]) @ V.T
    if noise:
        rng_n = np.random.default_rng([seed, 3])
        A = A + noise * rng_n.standard_normal((N, n))
    At = torch.from_numpy(np.asfortranarray(A))
    return as_colmajor(At.to(dtype)).to(device)


def dct_lowrank(N: int, n: int, sigma: np.ndarray, seed: int,
                dtype=torch.float32, device="cpu") -> torch.Tensor:
    """A = U diag(sigma) V^T with exactly orthonormal U built from n distinct
    DCT-II columns (random frequencies, random signs, random row permutation)
    and V from QR of a seeded n x n Gaussian.  O(N n) work to form U."""
    rng = np.random.default_rng([seed, 7])
    freqs = np.sort(rng.choice(N, size=n, replace=False))
    signs = rng.choice([-1.0, 1.0], size=n)
    perm = torch.from_numpy(rng.permutation(N))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    dev = torch.device(device)
    i = torch.arange(N, dtype=torch.float64, device=dev)
    f = torch.tensor(freqs, dtype=torch.float64, device=dev)
    scale = torch.where(f == 0, math.sqrt(1.0 / N), math.sqrt(2.0 / N))
    U = torch.cos(math.pi * (i[:, None] + 0.5) * f[None, :] / N) * scale[None, :]
    U = U * torch.tensor(signs, dtype=torch.float64, device=dev)[None, :]
    U = U[perm.to(dev)]
    SVt = torch.tensor(np.asarray(sigma, dtype=np.float64)[:, None] * V.T, device=dev)
    A = U @ SVt
    out = colmajor_empty(N, n, dtype, dev)
    out.copy_(A)
    return out


def batched_shapes(count: int = 64, seed: int = 4004) -> list:
    """Shapes of the uneven batch: (N, n, k) per matrix with N log-uniform in
    [16384, 1048576], n uniform in [64, 512] and k uniform in [8, 64]."""
    rng = np.random.default_rng(seed)
    N = np.rint(np.exp(rng.uniform(math.log(16384), math.log(1048576), count))).astype(np.int64)
    n = rng.integers(64, 513, count)
    k = rng.integers(8, 65, count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(N, n, k)]


def batched_matrix(N: int, n: int, seed: int, device="cpu", ld_multiple: int = 4) -> torch.Tensor:
    """One matrix of the uneven batch: sigma_j = j^-1.5 (j = 1 .. n) on
    DCT-based orthonormal factors (``dct_lowrank``), FP32, column-major with
    the leading dimension rounded up to ``ld_multiple`` (16-byte aligned
    columns)."""
    sigma = np.arange(1, n + 1, dtype=np.float64) ** -1.5
    A = dct_lowrank(N, n, sigma, seed, dtype=torch.float32, device=device)
    ld = (N + ld_multiple - 1) // ld_multiple * ld_multiple
    if ld == N:
        return A
    store = torch.zeros((n, ld), dtype=torch.float32, device=A.device)
    out = store[:, :N].T
    out.copy_(A)
    return out


def coarse_rows_every_other(nx: int, ny: int, nz: int, ncomp: int = 3) -> np.ndarray:
    """Row indices of the grid points with even (i, j, k) in every component
    (2x sub-sampling per dimension, "direct injection"), sorted ascending."""
    c = np.arange(ncomp)[:, None, None, None]
    i = np.arange(0, nx, 2)[None, :, None, None]
    j = np.arange(0, ny, 2)[None, None, :, None]
    k = np.arange(0, nz, 2)[None, None, None, :]
    rows = ((c * nx + i) * ny + j) * nz + k
    return np.sort(rows.reshape(-1)).astype(np.int64)


@dataclass(frozen=True)
class StructuredMesh:
    """A tensor-product grid and a coarse subset of it, described as input
    data only (coordinates and index lists; no interpolation weights).

    Rows of a field on this grid are ordered ((c * nx + i) * ny + j) * nz + k
    for component c, x index i, y index j, z index k (z fastest), as in
    ``spectral_snapshots``.  ``coarse[d]`` lists the kept indices of
    dimension d (strictly increasing); ``period[d] > 0`` marks dimension d as
    periodic with that period (0: bounded)."""
    ncomp: int
    n: tuple
    coords: tuple
    coarse: tuple
    period: tuple

    @property
    def rows(self) -> int:
        return self.ncomp * self.n[0] * self.n[1] * self.n[2]

    @property
    def coarse_rows(self) -> np.ndarray:
        """Global row indices of the coarse grid points, sorted ascending."""
        nx, ny, nz = self.n
        cx, cy, cz = (np.asarray(c, np.int64) for c in self.coarse)
        c = np.arange(self.ncomp, dtype=np.int64)[:, None, None, None]
        r = ((c * nx + cx[None, :, None, None]) * ny + cy[None, None, :, None]) * nz \
            + cz[None, None, None, :]
        return r.reshape(-1)


def channel_mesh(cfg: SpectralConfig, stride=(2, 2, 2), periodic: bool = False,
                 keep_last: bool = False) -> StructuredMesh:
    """The grid of ``spectral_snapshots`` (uniform x and z, wall-clustered y)
    with every stride-th point kept per dimension (indices 0, s, 2s, ...;
    with ``keep_last`` the last index is added when the stride skips it).
    ``periodic`` marks x and z periodic with the box lengths."""
    x = np.arange(cfg.nx, dtype=np.float64) * (cfg.lx / cfg.nx)
    y = -np.cos(np.pi * np.arange(cfg.ny, dtype=np.float64) / max(cfg.ny - 1, 1))
    z = np.arange(cfg.nz, dtype=np.float64) * (cfg.lz / cfg.nz)
    coarse = []
    for n_d, s in zip((cfg.nx, cfg.ny, cfg.nz), stride):
        idx = list(range(0, n_d, s))
        if keep_last and idx[-1] != n_d - 1:
            idx.append(n_d - 1)
        coarse.append(np.asarray(idx, np.int64))
    period = (cfg.lx, 0.0, cfg.lz) if periodic else (0.0, 0.0, 0.0)
    return StructuredMesh(3, (cfg.nx, cfg.ny, cfg.nz), (x, y, z), tuple(coarse), period)
