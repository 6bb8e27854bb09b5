"""Vector-mode extraction on the GPU (sec. 6.2) against the oracle: the 3-D
FFT element by element against numpy's, and the shell spectra (mean |k|,
mode count, P_curl, P_div, P_vector, P_scalar) against oracle.spectra on the
same inputs: random fields, a plane wave, and the shift, B^i and momentum
density of a solved Zel'dovich step; at 256^3 with 32 shells (a quarter of
Nyquist).

Tolerances: FP64 transforms of n^3 points carry a rounding error of order
log2(n^3) eps relative to the largest mode; per shell the sums are over
thousands of modes in a different order from numpy's, so each spectrum row
is compared to 1e-11 of that shell's total power (P_curl + P_div, or P_vector
+ P_scalar), the mode counts exactly, and |k| to 1e-13.
"""
import numpy as np
import pytest

from oracle import spectra as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1905_08890_amd import grmg, synth  # noqa: E402


def _fields(n, seed):
    r = np.random.default_rng(seed)
    return [r.standard_normal((n, n, n)) for _ in range(3)]


def _compare(got, ref):
    assert got.shape == ref.shape
    assert np.array_equal(got[1], ref[1]), (got[1], ref[1])
    assert np.allclose(got[0], ref[0], rtol=1e-13, atol=0)
    tot_cd = ref[2] + ref[3]
    tot_vs = ref[4] + ref[5]
    for r, tot in ((2, tot_cd), (3, tot_cd), (4, tot_vs), (5, tot_vs)):
        err = np.abs(got[r] - ref[r])
        assert np.all(err <= 1e-11 * tot), (r, err.max(), tot.min())


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_fft_matches_numpy(n):
    print(f"[spectra] fft n={n}", flush=True)
    r = np.random.default_rng(n)
    a = r.standard_normal((n, n, n)) + 1j * r.standard_normal((n, n, n))
    S = grmg.Spectra(n, nbins=max(1, n // 8))
    d = torch.from_numpy(a.copy()).cuda()
    S.fft(d)
    ref = np.fft.fftn(a)
    err = np.abs(d.cpu().numpy() - ref).max()
    assert err <= 4 * np.log2(n ** 3) * 2.2e-16 * np.abs(ref).max(), err
    S.close()


@pytest.mark.parametrize("n,nbins,seed", [(16, 2, 1), (32, 4, 2), (32, 8, 3), (64, 8, 4), (64, 16, 5)])
def test_random_field_spectra_match_oracle(n, nbins, seed):
    print(f"[spectra] random n={n} nbins={nbins}", flush=True)
    v = _fields(n, seed)
    S = grmg.Spectra(n, nbins)
    got = S.vector(*[torch.from_numpy(a).cuda() for a in v])
    _compare(got, OS.vector_spectra(*v, nbins=nbins))
    # a second call on other data reuses the handle
    w = _fields(n, seed + 100)
    _compare(S.vector(*[torch.from_numpy(a).cuda() for a in w]), OS.vector_spectra(*w, nbins=nbins))
    S.close()


def test_plane_wave_and_pure_modes():
    n, m0, A = 32, 3, 0.7
    c = np.arange(n) / n
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    z = np.zeros((n, n, n))
    S = grmg.Spectra(n, 4)
    got = S.vector(*[torch.from_numpy(a).cuda() for a in (z, A * np.cos(2 * np.pi * m0 * X), z)])
    keff = n * np.sin(2 * np.pi * m0 / n)
    assert np.isclose(got[2, 2] * got[1, 2], A * A * keff * keff / 2, rtol=1e-12)
    assert np.isclose(got[4, 2] * got[1, 2], A * A / 2, rtol=1e-12)
    # the divergence is zero in every cell, but it shares a complex transform with
    # curl_z, so its separated transform carries that transform's rounding (~eps)
    assert np.all(got[3] <= 1e-28 * got[2].max())
    # a gradient has no vector mode, a curl no scalar mode (to rounding)
    phi = _fields(n, 7)[0]
    g = [OS._d(phi, ax) for ax in (2, 1, 0)]
    got = S.vector(*[torch.from_numpy(a).cuda() for a in g])
    assert np.all(got[2] <= 1e-24 * got[3])
    cu = OS.curl_div(*_fields(n, 8))[:3]
    got = S.vector(*[torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in cu])
    assert np.all(got[3] <= 1e-24 * got[2])
    S.close()


def test_solved_shift_and_momentum_spectra_match_oracle():
    """beta^i, B^i and s_i of a solved 64^3 Zel'dovich step: GPU spectra equal
    the oracle's on the same arrays; beta's scalar mode dominates its vector
    mode on the largest scales (sec. 6.2; the Zel'dovich velocities are
    irrotational, so the vector mode comes from the density-velocity product
    and the deposit only)."""
    n = 64
    print("[spectra] solved 64^3 step", flush=True)
    pos, u, mass = synth.zeldovich(n, 1, 0.3)
    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE)
    g.deposit_sources(torch.from_numpy(pos).cuda(), torch.from_numpy(u).cuda(), mass)
    rep = g.solve_constraints(rtol=1e-10)
    assert rep["status"] == grmg.OK
    S = grmg.Spectra(n)
    for ids in ((grmg.BETAX, grmg.BETAY, grmg.BETAZ), (grmg.BX, grmg.BY, grmg.BZ), (grmg.SX, grmg.SY, grmg.SZ)):
        f = [g.get_field(i).clone() for i in ids]
        got = S.vector(*f)
        ref = OS.vector_spectra(*[t.cpu().numpy() for t in f], nbins=n // 8)
        _compare(got, ref)
        print(f"[spectra] fields {ids}: shell 0 P_vector {got[4, 0]:.3e} P_scalar {got[5, 0]:.3e}", flush=True)
        if ids[0] == grmg.BETAX:
            assert got[5, 0] > got[4, 0], got[4:, 0]
    S.close()
    g.close()


def test_full_size_256_with_32_shells():
    n = 256
    print("[spectra] 256^3, 32 shells", flush=True)
    r = np.random.default_rng(11)
    v = [synth.grf(n, 20 + i, -2.0, 1.0) + 0.1 * r.standard_normal((n, n, n)) for i in range(3)]
    S = grmg.Spectra(n, 32)
    got = S.vector(*[torch.from_numpy(a).cuda() for a in v])
    _compare(got, OS.vector_spectra(*v, nbins=32))
    S.close()
