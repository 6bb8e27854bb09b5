"""Pins of the oracle's vector-mode extraction (sec. 6.2: discrete curl, and
power spectra of the vector and scalar modes up to a quarter of Nyquist)
against facts fixed independently of its code:

* a plane wave has a closed-form curl spectrum (one shell, known amplitude);
* the central-difference curl of a central-difference gradient and the
  divergence of a central-difference curl vanish (the differences commute);
* per mode, |k x v|^2 + |k . v|^2 = |k|^2 |v|^2 (Lagrange's identity), so the
  vector- plus scalar-mode power of a field is its total power, computed here
  straight from the field's own transform;
* shell counts and mean |k| by brute-force enumeration of integer vectors;
* an explicit triple-sum DFT on a tiny grid.
"""
import itertools

import numpy as np

from oracle import spectra as S


def _rng_field(n, seed):
    r = np.random.default_rng(seed)
    return [r.standard_normal((n, n, n)) for _ in range(3)]


def _coords(n):
    c = np.arange(n) / n
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return X, Y, Z


def test_plane_wave_closed_form():
    """v = (0, A cos(2 pi m0 x), 0): the curl is z-directed, -A sin(2 pi m0 x)
    k_eff; all its power sits in the two modes (+-m0, 0, 0) of shell m0 - 1,
    P_curl = A^2 k_eff^2 / 4 each, P_vector = A^2 / 4 each; no divergence."""
    n, m0, A = 32, 3, 0.7
    X, _, _ = _coords(n)
    z = np.zeros((n, n, n))
    out = S.vector_spectra(z, A * np.cos(2 * np.pi * m0 * X), z, nbins=4)
    keff = n * np.sin(2 * np.pi * m0 / n)
    b = m0 - 1
    assert np.isclose(out[2, b] * out[1, b], A * A * keff * keff / 2, rtol=1e-12)
    assert np.isclose(out[4, b] * out[1, b], A * A / 2, rtol=1e-12)
    assert np.all(out[3] == 0.0) and np.all(out[5] == 0.0)
    others = [j for j in range(4) if j != b]
    assert np.all(out[2, others] < 1e-28 * out[2, b])


def test_gradient_has_no_curl_and_curl_has_no_divergence():
    n = 24
    phi = _rng_field(n, 1)[0]
    g = [S._d(phi, ax) for ax in (2, 1, 0)]
    out = S.vector_spectra(*g, nbins=3)
    assert np.all(out[3] > 0)
    assert np.all(out[2] < 1e-26 * out[3])
    A = _rng_field(n, 2)
    c = S.curl_div(*A)[:3]
    out = S.vector_spectra(*c, nbins=3)
    assert np.all(out[2] > 0)
    assert np.all(out[3] < 1e-26 * out[2])


def test_vector_plus_scalar_mode_power_is_total_power():
    """Per shell, count * (P_vector + P_scalar) equals the summed power of v's
    own components over the shell's modes (rtol 1e-12)."""
    n = 32
    v = _rng_field(n, 3)
    out = S.vector_spectra(*v, nbins=4)
    N = float(n) ** 3
    pv = sum(np.abs(np.fft.fftn(c)) ** 2 for c in v) / N ** 2
    m = np.fft.fftfreq(n, 1.0 / n)
    mz, my, mx = np.meshgrid(m, m, m, indexing="ij")
    mag = np.sqrt(mx ** 2 + my ** 2 + mz ** 2)
    for b in range(4):
        sel = (mag >= b + 0.5) & (mag < b + 1.5)
        assert np.isclose(out[1, b] * (out[4, b] + out[5, b]), pv[sel].sum(), rtol=1e-12)
        # the vector and scalar parts are each a real share (both strictly positive for a random field)
        assert out[4, b] > 0 and out[5, b] > 0


def test_shell_counts_and_mean_k_by_enumeration():
    n, nb = 12, 3
    counts = [0] * nb
    ksum = [0.0] * nb
    half = n // 2
    for m in itertools.product(range(-half, half), repeat=3):
        r = (m[0] ** 2 + m[1] ** 2 + m[2] ** 2) ** 0.5
        for b in range(nb):
            if b + 0.5 <= r < b + 1.5:
                counts[b] += 1
                ksum[b] += 2 * np.pi * r
    out = S.vector_spectra(*_rng_field(n, 4), nbins=nb)
    assert list(out[1].astype(int)) == counts
    assert counts[0] == 18        # 6 face neighbours and 12 edge neighbours (|m| = 1, sqrt 2)
    assert np.allclose(out[0], np.array(ksum) / np.array(counts), rtol=1e-14)


def test_tiny_grid_against_explicit_dft():
    """n = 6: the shell-0 mean of P_curl and P_div from triple-sum DFTs of
    the curl and divergence computed point by point."""
    n = 6
    v = _rng_field(n, 5)
    h = 1.0 / n

    def at(f, z, y, x):
        return f[z % n, y % n, x % n]

    cur = np.zeros((4, n, n, n))
    for z, y, x in itertools.product(range(n), repeat=3):
        d = lambda f, dz, dy, dx: (at(f, z + dz, y + dy, x + dx) - at(f, z - dz, y - dy, x - dx)) / (2 * h)
        vx, vy, vz = v
        cur[0, z, y, x] = d(vz, 0, 1, 0) - d(vy, 1, 0, 0)
        cur[1, z, y, x] = d(vx, 1, 0, 0) - d(vz, 0, 0, 1)
        cur[2, z, y, x] = d(vy, 0, 0, 1) - d(vx, 0, 1, 0)
        cur[3, z, y, x] = d(vx, 0, 0, 1) + d(vy, 0, 1, 0) + d(vz, 1, 0, 0)
    N = n ** 3
    pc, pd, cnt = 0.0, 0.0, 0
    for m in itertools.product(range(-3, 3), repeat=3):
        r = np.sqrt(sum(q * q for q in m))
        if not (0.5 <= r < 1.5):
            continue
        cnt += 1
        F = np.zeros(4, dtype=complex)
        for z, y, x in itertools.product(range(n), repeat=3):
            F += cur[:, z, y, x] * np.exp(-2j * np.pi * (m[0] * z + m[1] * y + m[2] * x) / n)
        pc += float((np.abs(F[:3]) ** 2).sum()) / N ** 2
        pd += float(np.abs(F[3]) ** 2) / N ** 2
    out = S.vector_spectra(*v, nbins=1)
    assert out[1, 0] == cnt == 18
    assert np.isclose(out[2, 0], pc / cnt, rtol=1e-12)
    assert np.isclose(out[3, 0], pd / cnt, rtol=1e-12)
