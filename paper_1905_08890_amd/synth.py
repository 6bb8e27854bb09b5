"""Seeded synthetic workloads shared by the GPU path's tests/benchmarks and the
CPU oracle.

This module holds no arithmetic of the method itself (no deposit, no
operator, no solver): only random fields and particle sets with the shapes,
spectra and sizes of the paper's workloads.  The paper's own initial
conditions (modified CAMB + 2LPTic, sec. 7) are not available, so these
stand in for them:

* ``grf(n, seed, p, sigma)``: Gaussian random field on n^3 with power
  spectrum P(k) ~ k^p (k = 2 pi |integer wavevector|, k = 0 removed),
  zero mean, rescaled to standard deviation ``sigma``.
* ``zeldovich(n, seed, rms_cells)``: n^3 equal-mass particles displaced from
  the cell centres of an n^3 lattice by a longitudinal Gaussian displacement
  d = -grad(phi) with P_d(k) ~ k^-3, scaled to rms |d| = rms_cells / n, with
  lower-index momenta u = lam * d and mass 1/n^3 (so <s0> is about 1).
"""
from __future__ import annotations

import numpy as np

OMEGA_M = 0.3072                      # Planck-like value used in sec. 6
C_TILDE = 2997.92458 / 256.0          # c/(L H0) for L = 256 Mpc/h (sec. 5.1)


def _kgrid(n):
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    kr = 2.0 * np.pi * np.fft.rfftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, kr, indexing="ij")
    return kz, ky, kx


def grf(n: int, seed: int, p: float, sigma: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    W = np.fft.rfftn(w)
    kz, ky, kx = _kgrid(n)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = 1.0
    W *= k ** (p / 2.0)
    W[0, 0, 0] = 0.0
    d = np.fft.irfftn(W, s=(n, n, n), axes=(0, 1, 2))
    d -= d.mean()
    d *= sigma / d.std()
    return np.ascontiguousarray(d)


def zeldovich(n: int, seed: int, rms_cells: float, lam: float = 1.0):
    """Returns (pos[n^3,3] in [0,1), u[n^3,3], mass); columns are (x, y, z)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    W = np.fft.rfftn(w)
    kz, ky, kx = _kgrid(n)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = 1.0
    phik = W * k ** (-5.0 / 2.0)          # potential with P_phi ~ k^-5
    phik[0, 0, 0] = 0.0
    # drop the Nyquist planes so that the odd derivative stays real
    nyq = n // 2
    phik[nyq, :, :] = 0.0
    phik[:, nyq, :] = 0.0
    phik[:, :, -1] = 0.0
    disp = [np.fft.irfftn(-1j * kk * phik, s=(n, n, n), axes=(0, 1, 2)) for kk in (kx, ky, kz)]
    rms = np.sqrt(np.mean(disp[0] ** 2 + disp[1] ** 2 + disp[2] ** 2))
    scale = (rms_cells / n) / rms
    h = 1.0 / n
    cz, cy, cx = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    pos = np.empty((n ** 3, 3))
    u = np.empty((n ** 3, 3))
    for c, (cc, dd) in enumerate(zip((cx, cy, cz), disp)):
        d = (dd * scale).ravel()
        pos[:, c] = np.mod(cc.ravel() * h + d, 1.0)
        u[:, c] = lam * d
    pos[pos >= 1.0] = 0.0                  # np.mod can round up to exactly 1.0
    return np.ascontiguousarray(pos), np.ascontiguousarray(u), 1.0 / n ** 3


def hamiltonian_only_sources(n: int = 32, seed: int = 0, sigma: float = 0.1):
    """32^3 Hamiltonian-only workload: s0 = 1 + delta, delta a k^-2 GRF;
    s_i = s_m = 0.  Returns (s0, sx, sy, sz, sm)."""
    s0 = 1.0 + grf(n, seed, -2.0, sigma)
    z = np.zeros((n, n, n))
    return s0, z, z.copy(), z.copy(), z.copy()


WORKLOADS = {
    # name: (grid side, particle seed, rms displacement in cells)
    "zeldovich128": (128, 1, 0.3),
    "zeldovich256": (256, 2, 1.0),
}


BATCH_SIDES = (32, 48, 64, 96, 128)


def batch_item(seed: int, sides=BATCH_SIDES, sigma_range=(0.05, 1.0)):
    """One box of the batched workload: side drawn from `sides`, density
    contrast sigma log-uniform in sigma_range, delta a k^-2 GRF (seed `seed`),
    s0 = 1 + delta, longitudinal momentum s_i = -d_i Lap^-1 delta rescaled to
    rms |s| = 1e-3, s_m = 0.  Returns (n, (s0, sx, sy, sz, sm))."""
    rng = np.random.default_rng(seed)
    n = int(rng.choice(np.asarray(sides)))
    sigma = float(np.exp(rng.uniform(np.log(sigma_range[0]), np.log(sigma_range[1]))))
    return n, _matter_sources(n, seed, sigma)


def _matter_sources(n: int, seed: int, sigma: float):
    """s0 = 1 + delta (k^-2 GRF of std sigma), longitudinal momentum
    -d_i Lap^-1 delta rescaled to rms |s| = 1e-3, s_m = 0."""
    delta = grf(n, seed, -2.0, sigma)
    D = np.fft.fftn(delta)
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    mom = [np.real(np.fft.ifftn(1j * kk / k2 * D)) for kk in (kx, ky, kz)]
    rms = np.sqrt(np.mean(mom[0] ** 2 + mom[1] ** 2 + mom[2] ** 2))
    mom = [np.ascontiguousarray(m * (1e-3 / rms)) for m in mom]
    return (1.0 + delta, mom[0], mom[1], mom[2], np.zeros((n, n, n)))


PATCH_SIDES = tuple(range(24, 81, 8))


def patch_item(j: int, box_sides, first_seed: int = 196, sides=PATCH_SIDES, sigma_range=(0.05, 1.0)):
    """Refinement patch j of the batched workload (seed first_seed + j): side
    from `sides`, spacing half its parent's, parent = the first box from box j
    on (cyclically) with n_parent >= side/2 + 4, lower corner at a random
    whole parent cell, its own sources as for a box (sigma log-uniform).
    box_sides: the periodic boxes' sides (unit boxes).  Returns
    ((n, h, parent, origin), (s0, sx, sy, sz, sm))."""
    seed = first_seed + j
    rng = np.random.default_rng(seed)
    n = int(rng.choice(np.asarray(sides)))
    sigma = float(np.exp(rng.uniform(np.log(sigma_range[0]), np.log(sigma_range[1]))))
    nb = len(box_sides)
    parent = next((b % nb for b in range(j, j + nb) if box_sides[b % nb] >= n // 2 + 4), None)
    if parent is None:
        raise ValueError(f"no box can hold a patch of side {n}")
    N = box_sides[parent]
    H = 1.0 / N
    span = N - n // 2
    off = [int(rng.integers(2, span - 1)) if span > 4 else 0 for _ in range(3)]
    return (n, H / 2.0, parent, tuple(o * H for o in off)), _matter_sources(n, seed, sigma)


def zeldovich_trajectory(n: int, seed: int, rms_cells_list, lam: float = 1.0):
    """The same Zel'dovich displacement pattern (seed) at a sequence of rms
    amplitudes: a growing trajectory standing in for consecutive time steps.
    Yields (pos, u, mass) per amplitude; the FFTs are done once."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    W = np.fft.rfftn(w)
    kz, ky, kx = _kgrid(n)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    k[0, 0, 0] = 1.0
    phik = W * k ** (-5.0 / 2.0)
    phik[0, 0, 0] = 0.0
    nyq = n // 2
    phik[nyq, :, :] = 0.0
    phik[:, nyq, :] = 0.0
    phik[:, :, -1] = 0.0
    disp = [np.fft.irfftn(-1j * kk * phik, s=(n, n, n), axes=(0, 1, 2)).ravel() for kk in (kx, ky, kz)]
    rms = np.sqrt(np.mean(disp[0] ** 2 + disp[1] ** 2 + disp[2] ** 2))
    h = 1.0 / n
    cz, cy, cx = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    centres = [c.ravel() * h for c in (cx, cy, cz)]
    for r in rms_cells_list:
        scale = (r / n) / rms
        pos = np.empty((n ** 3, 3))
        u = np.empty((n ** 3, 3))
        for c in range(3):
            d = disp[c] * scale
            pos[:, c] = np.mod(centres[c] + d, 1.0)
            u[:, c] = lam * d
        pos[pos >= 1.0] = 0.0
        yield pos, u, 1.0 / n ** 3
