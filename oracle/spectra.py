"""FP64 CPU reference of the vector-mode extraction (test infrastructure only).

Paper sec. 6.2 (the shift-vector power spectrum): the shift beta^i (and B^i,
and the momentum density s_i that sources it) mixes a scalar and a vector
mode; a discrete curl removes the scalar part, and the vector mode's power
follows from k^2 P_{beta^V}(k) = P_{curl beta}(k).  Spectra are shown up to a
quarter of the Nyquist frequency.

What this module computes, for three real fields v_x, v_y, v_z on the
periodic unit box (n^3 cells, h = 1/n, arrays [z][y][x], x fastest):

* the discrete curl and divergence with 3-point central differences (the
  same differences the paper's code uses for gradients);
* their Fourier transforms F[g](m) = sum_x g(x) exp(-2 pi i m.x) (numpy's FFT
  as the library step), for integer wave vectors m, k = 2 pi m;
* per mode: P_curl = sum_i |F[(curl v)_i]|^2 / N^2 and P_div = |F[div v]|^2 /
  N^2 (N = n^3; box volume 1), and the vector- and scalar-mode power of v
  itself, P_vector = P_curl / |k_eff|^2 and P_scalar = P_div / |k_eff|^2,
  with k_eff,i = sin(2 pi m_i / n) n, the Fourier symbol of the central
  difference (so that P_vector + P_scalar is exactly the power of v per mode,
  the discrete form of k^2 P_V = P_curl);
* shells: bin j (0 <= j < nbins) holds the modes with j + 1/2 <= |m| < j + 3/2,
  i.e. centred on |k| = 2 pi (j + 1); the default nbins = n / 8 reaches a
  quarter of the Nyquist wave number pi n.

Per bin it returns the mode count, the mean |k|, and the means of P_curl,
P_div, P_vector and P_scalar over the bin's modes.  Readings where the paper
is silent (the difference stencil, the shell edges, the normalisation) are
the ones stated here.
"""
from __future__ import annotations

import numpy as np

ROWS = ("k", "count", "p_curl", "p_div", "p_vector", "p_scalar")


def _d(f, axis):
    """Central difference along an array axis (2 = x, 1 = y, 0 = z), periodic, h = 1/n."""
    n = f.shape[axis]
    return (np.roll(f, -1, axis) - np.roll(f, 1, axis)) * (0.5 * n)


def curl_div(vx, vy, vz):
    """(curl_x, curl_y, curl_z, div) of v by central differences."""
    dx = lambda f: _d(f, 2)
    dy = lambda f: _d(f, 1)
    dz = lambda f: _d(f, 0)
    cx = dy(vz) - dz(vy)
    cy = dz(vx) - dx(vz)
    cz = dx(vy) - dy(vx)
    div = dx(vx) + dy(vy) + dz(vz)
    return cx, cy, cz, div


def wavenumbers(n):
    """Integer wave vectors (mz, my, mx) of the FFT's output order, each in [-n/2, n/2)."""
    m = np.fft.fftfreq(n, 1.0 / n)
    return np.meshgrid(m, m, m, indexing="ij")


def shell_index(mz, my, mx):
    """Bin of each mode: floor(|m| + 1/2) - 1 (the k = 0 mode gets -1)."""
    return np.floor(np.sqrt(mx * mx + my * my + mz * mz) + 0.5).astype(np.int64) - 1


def mode_powers(vx, vy, vz):
    """Per-mode P_curl, P_div, |k_eff|^2 and the integer wave vectors."""
    n = vx.shape[0]
    N = float(n) ** 3
    cx, cy, cz, div = curl_div(vx, vy, vz)
    p_curl = sum(np.abs(np.fft.fftn(c)) ** 2 for c in (cx, cy, cz)) / N ** 2
    p_div = np.abs(np.fft.fftn(div)) ** 2 / N ** 2
    mz, my, mx = wavenumbers(n)
    keff2 = sum((n * np.sin(2.0 * np.pi * m / n)) ** 2 for m in (mx, my, mz))
    return p_curl, p_div, keff2, (mz, my, mx)


def vector_spectra(vx, vy, vz, nbins=None):
    """[6][nbins] array: rows ROWS (k, count, P_curl, P_div, P_vector, P_scalar) per shell."""
    n = vx.shape[0]
    if nbins is None:
        nbins = n // 8
    p_curl, p_div, keff2, (mz, my, mx) = mode_powers(vx, vy, vz)
    j = shell_index(mz, my, mx)
    mag = np.sqrt(mx * mx + my * my + mz * mz)
    out = np.zeros((6, nbins))
    for b in range(nbins):
        sel = j == b
        c = int(sel.sum())
        out[1, b] = c
        if c == 0:
            continue
        out[0, b] = 2.0 * np.pi * mag[sel].mean()
        out[2, b] = p_curl[sel].mean()
        out[3, b] = p_div[sel].mean()
        out[4, b] = (p_curl[sel] / keff2[sel]).mean()
        out[5, b] = (p_div[sel] / keff2[sel]).mean()
    return out
