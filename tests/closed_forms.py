"""Closed forms used to pin the oracle: discrete Fourier symbols of the
paper's finite-difference operators and exact FFT solves of the linear
problems.  Written from the mathematics, independent of oracle/ and of the
GPU library."""
import numpy as np


def centres(n):
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def kvec(n):
    """Integer wavenumbers times 2 pi, full complex FFT layout, axes (z, y, x)."""
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    return KX, KY, KZ


def lap_symbol(n):
    """Eigenvalue of the 7-point Laplacian on exp(i k.x): -(4/h^2) sum sin^2(k_d h/2)."""
    h = 1.0 / n
    KX, KY, KZ = kvec(n)
    return -(4.0 / h ** 2) * (np.sin(KX * h / 2) ** 2 + np.sin(KY * h / 2) ** 2 + np.sin(KZ * h / 2) ** 2)


def dcen_symbol(n, axis):
    """Symbol of the central difference (g(x+h)-g(x-h))/2h: i sin(k h)/h."""
    h = 1.0 / n
    K = kvec(n)[axis]
    return 1j * np.sin(K * h) / h


def helmholtz_fft(f, mu2):
    """Zero-mean solution of Lap_h phi - mu2 phi = f - <f> (exact)."""
    n = f.shape[0]
    F = np.fft.fftn(f)
    den = lap_symbol(n) - mu2
    F[0, 0, 0] = 0.0
    den[0, 0, 0] = 1.0
    return np.real(np.fft.ifftn(F / den))


def apply_symbol(g, sym):
    return np.real(np.fft.ifftn(np.fft.fftn(g) * sym))


def roll_lap(p):
    n = p.shape[0]
    return (sum(np.roll(p, s, ax) for ax in range(3) for s in (1, -1)) - 6.0 * p) * n * n


def maxrel(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))
