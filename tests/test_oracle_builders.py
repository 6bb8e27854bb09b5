"""Pins of the oracle's two nonlinear source builders against the paper's
equations in their *physical* (sec. 2) form and in the paper's own variables
psi and alpha, not against the code-unit formulas the builders restate.

* CMC coefficient m^2 and source f (builder of the xi equation, sec. 4.3.2.2):
  derived symbolically here from the sec. 2 lapse equation for alpha psi under
  CMC slicing, with the sec. 2 Hamiltonian constraint and the code-unit
  Friedmann equations of sec. 4.1.1 used to remove K^2 and dK/dt, then
  converted by the code-unit scalings of sec. 4.1.1 (G = c = 1 in sec. 2,
  c~ = 1/(L H0)).  The builders must reproduce the resulting coefficient of xi
  and the xi-free part to rounding at random points, for a != 1 and c~ = O(1).
  A reading: the sec. 2 equations are taken with Omega_Lambda = 0 and a cold
  background (no homogeneous pressure), where the printed Lambda terms of the
  lapse equation and of the second Friedmann equation play no part; the
  builders take no Omega_Lambda, so these cases fix every coefficient they use.
  Also pinned by its linearisation about FLRW: the solved xi must approach the
  exact FFT Helmholtz solution of the linearised equation at second order.
* Shift source 2 d_j[alpha psi^-6 A^ij] a^3 (the MD-gauge equation in code
  units, sec. 4.1.1, whose vector Laplacian reduces to Lap B^i, sec. 4.3.1):
  the continuum divergence is differentiated symbolically in psi and alpha
  with smooth, strongly nonlinear fields (chi far from 1, a != 1, c~ = O(1));
  the builders' central differences must converge to it at second order.
Both checks are applied to the periodic oracle and to the patch oracle.
"""
import numpy as np
import pytest
import sympy as sp

import oracle as O
from oracle import dirichlet as D
from closed_forms import centres, helmholtz_fft, maxrel
from paper_1905_08890_amd import synth


# ------------------------------------------------- the lapse equation (sec. 2)

def _cmc_from_physical_equations():
    """Returns (m2, f) as functions of (Psi, s0, s, AA; a, Om, c) from the
    sec. 2 form of the CMC lapse equation.

    Pointwise unknowns (code units): Psi, xi = Phi chi, their Laplacians, the
    stress trace s and A_ijA^ij; Lap Psi follows from s0 by the Hamiltonian
    constraint.  The CMC residual times a^2 c^2 L^2 / a^(1/2) is affine in xi
    and Lap xi; evaluated numerically it must read Lap xi - m2 xi - f, which
    defines m2 and f (checked: unit slope in Lap xi, no dependence on L)."""
    a, Om, c, L = sp.symbols("a Om c L", positive=True)
    Psi, xi, lapPsi, lapxi, AAt, st, s0t = sp.symbols("Psi xi lapPsi lapxi AAt st s0t", real=True)
    H0 = 1 / (c * L)                        # c~ = c/(L H0) with c = 1
    rho_c = 3 * H0 ** 2 / (8 * sp.pi)       # critical density, G = 1
    rho_m = Om * rho_c / a ** 3             # homogeneous matter, code density 1
    # code-unit Friedmann equations (sec. 4.1.1) at Omega_Lambda = 0, S^ = 0:
    Kt2 = 12 * a ** 4 * sp.Rational(3, 4) * Om / a ** 3          # K~^2
    dKt = a ** 2 * (Kt2 / (3 * a ** 4) + sp.Rational(3, 2) * Om / a ** 3)   # d(a^-2 K~)/dt~
    # back to physical K (K~ = a^2 c~ L K) and dK/dt (dt~ = H0 dt / a^2)
    K2 = Kt2 / (a ** 2 * c * L) ** 2
    Kdot = H0 / (a ** 2 * c * L) * dKt
    # code-unit variables -> physical (sec. 4.1.1 scalings)
    chi = 1 - Psi / (2 * a ** 2 * c ** 2)
    psi = sp.sqrt(a) * chi
    Phi = xi / chi
    alpha = 1 + Phi / (a ** 2 * c ** 2)
    s0 = Om * rho_c * s0t
    s = Om * rho_c * st
    AA = a ** 2 / (c ** 2 * L ** 2) * AAt
    lap_psi = sp.sqrt(a) * (-lapPsi / (2 * a ** 2 * c ** 2)) / L ** 2
    lap_alpha_psi = sp.sqrt(a) * (-lapPsi / (2 * a ** 2 * c ** 2) + lapxi / (a ** 2 * c ** 2)) / L ** 2
    # Hamiltonian constraint (sec. 2.4 step 2) ties Lap Psi to s0
    ham = sp.Eq(lap_psi, -2 * sp.pi / psi * s0 - psi ** -7 * AA / 8 + 2 * sp.pi * psi ** 5 * rho_m)
    lap_of_s0 = sp.solve(ham, lapPsi)[0]
    # lapse equation under CMC slicing (sec. 2.4 step 3), rho_Lambda = 0
    rhs = alpha * (2 * sp.pi / psi * (s0 + 2 * s) + sp.Rational(7, 8) * psi ** -7 * AA
                   + psi ** 5 * 5 * K2 / 12) - psi ** 5 * Kdot
    resid = ((lap_alpha_psi - rhs) * a ** 2 * c ** 2 * L ** 2 / sp.sqrt(a)).subs(lapPsi, lap_of_s0)
    R = sp.lambdify((Psi, xi, lapxi, AAt, st, s0t, a, Om, c, L), resid, "numpy")

    def parts(psi_, s0_, s_, AA_, a_, om_, c_):
        r = lambda x, lx, L_=1.7: R(psi_, x, lx, AA_, s_, s0_, a_, om_, c_, L_)
        r00 = r(0.0, 0.0)
        assert np.allclose(r(0.0, 1.0) - r00, 1.0, rtol=0, atol=1e-9)     # unit slope in Lap xi
        assert np.allclose(r(0.0, 0.0, 0.3), r00, rtol=1e-12, atol=1e-12)  # free of the length unit
        m2 = r00 - r(1.0, 0.0)
        assert np.allclose(r(2.0, 0.0), r00 - 2.0 * m2, rtol=1e-12, atol=1e-12)   # affine in xi
        return m2, -r00

    return parts


@pytest.fixture(scope="module")
def cmc_physical():
    return _cmc_from_physical_equations()


@pytest.mark.parametrize("a,om,c", [(0.7, 0.3, 1.3), (1.0, 0.3072, 11.710643), (0.25, 0.9, 0.6)])
def test_cmc_builder_equals_lapse_equation_of_sec2(cmc_physical, a, om, c):
    """m^2 and f of the periodic oracle and of the patch oracle equal the
    coefficient of xi and the xi-free part of the sec. 2 lapse equation, at
    random points with chi in [0.5, 1.5], s0, s and A_ijA^ij of order one."""
    parts = cmc_physical
    n = 6
    rng = np.random.default_rng(31)
    kap = 1.0 / (2 * a * a * c * c)
    chi = rng.uniform(0.5, 1.5, (n, n, n))
    psi = (1.0 - chi) / kap
    s0 = rng.uniform(0.2, 3.0, (n, n, n))
    sm = rng.uniform(0.0, 0.5, (n, n, n))
    AA = rng.uniform(0.0, 2.0, (n, n, n))
    prm = O.params(a=a, omega_m=om, c_tilde=c)
    M2, F = parts(psi, s0, sm, AA, a, om, c)
    m2, f = O.build_cmc(psi, s0, sm, AA, prm=prm)
    # rounding: chi^-7 at chi = 1/2 amplifies the last bits by ~10^2
    assert maxrel(m2, M2) < 1e-11
    assert maxrel(f, F) < 1e-11
    m2d, fd = D.build_cmc(psi, s0, sm, AA, prm)
    assert maxrel(m2d, M2) < 1e-11
    assert maxrel(fd, F) < 1e-11


def test_cmc_builder_separates_every_term(cmc_physical):
    """Each input moves m^2 and f as the sec. 2 equation says: with s, AA and
    Psi switched on one at a time the builders still agree, so no term can be
    compensated by another."""
    parts = cmc_physical
    a, om, c = 0.8, 0.35, 0.9
    prm = O.params(a=a, omega_m=om, c_tilde=c)
    n = 4
    rng = np.random.default_rng(32)
    base = dict(psi=np.zeros((n, n, n)), s0=np.ones((n, n, n)), sm=np.zeros((n, n, n)), AA=np.zeros((n, n, n)))
    kap = 1.0 / (2 * a * a * c * c)
    for key, val in (("psi", (1 - rng.uniform(0.6, 1.4, (n, n, n))) / kap), ("sm", rng.uniform(0, 1, (n, n, n))),
                     ("AA", rng.uniform(0, 1, (n, n, n))), ("s0", rng.uniform(0.1, 2, (n, n, n)))):
        args = dict(base)
        args[key] = val
        m2, f = O.build_cmc(args["psi"], args["s0"], args["sm"], args["AA"], prm=prm)
        M2, F = parts(args["psi"], args["s0"], args["sm"], args["AA"], a, om, c)
        assert np.abs(m2 - M2).max() <= 1e-12 * np.abs(M2).max(), key
        assert np.abs(f - F).max() <= 1e-12 * max(np.abs(F).max(), 1.0), key


def test_cmc_linearised_about_flrw_is_helmholtz():
    """s0 = 1 + eps delta, s = A_ijA^ij = 0: to first order Psi solves
    Lap Psi - mu^2 Psi = A eps delta and xi solves
    Lap xi - mu^2 xi = A (eps delta + 6 kappa Psi), mu^2 = 9 a Om kappa,
    A = 3/2 a Om (the FLRW limit of the lapse equation).  The oracle's xi
    (builder + solve) deviates from that FFT solution at second order: the
    relative deviation doubles when eps doubles."""
    n = 32
    prm = O.params(a=0.8, omega_m=0.3072, c_tilde=1.0)    # kappa ~ 0.8: the 6 kappa Psi term is visible
    kap = 1.0 / (2 * prm.a ** 2 * prm.c_tilde ** 2)
    A = 1.5 * prm.a * prm.omega_m
    mu2 = 9 * prm.a * prm.omega_m * kap
    delta = synth.grf(n, 41, -2.0, 1.0)
    z = np.zeros((n, n, n))
    devs = []
    for eps in (2e-3, 4e-3):
        s0 = 1.0 + eps * delta
        psi, st, _, _ = O.solve_equation(O.HAMILTONIAN, z, A * (s0 - 1.0), z, prm=prm, rtol=1e-13)
        assert st == O.OK
        m2, f = O.build_cmc(psi, s0, z, z, prm=prm)
        xi, st, _, _ = O.solve_equation(O.CMC, z, f, m2, prm=prm, rtol=1e-13)
        assert st == O.OK
        psi_lin = helmholtz_fft(A * eps * delta, mu2)
        xi_lin = helmholtz_fft(A * (eps * delta + 6 * kap * psi_lin), mu2)
        assert maxrel(xi_lin, helmholtz_fft(A * eps * delta, mu2)) > 1e-2   # the Psi feedback matters
        devs.append(maxrel(xi, xi_lin))
    assert devs[0] < 1e-2
    assert 1.8 < devs[1] / devs[0] < 2.2


# ------------------------------------------------- shift source (sec. 4.1.1)

def _shift_source_continuum(a, c):
    """Lambdified continuum 2 a^3 d_j(alpha psi^-6 A^ij) for fixed smooth
    periodic Psi, xi and A_ij on the unit box, plus the fields themselves."""
    x, y, z = sp.symbols("x y z", real=True)
    tp = 2 * sp.pi
    Psi = -0.9 * a * a * c * c * (sp.sin(tp * x) * sp.cos(tp * y) + 0.4 * sp.sin(tp * z + 0.3))
    xi = 0.5 * a * a * c * c * (sp.cos(tp * x + 0.2) + 0.6 * sp.sin(tp * y) * sp.sin(tp * z))
    A = {(0, 0): sp.sin(tp * y) + 0.3 * sp.cos(tp * z),
         (1, 1): sp.cos(tp * x) * sp.sin(tp * z),
         (2, 2): 0.7 * sp.sin(tp * (x + y)),
         (0, 1): sp.cos(tp * z) * sp.sin(tp * x),
         (0, 2): 0.5 * sp.sin(tp * y + 1.0),
         (1, 2): sp.cos(tp * (x - z))}
    for (i, j) in list(A):
        A[(j, i)] = A[(i, j)]
    chi = 1 - Psi / (2 * a * a * c * c)
    psi = sp.sqrt(a) * chi                   # psi = a^(1/2) (1 - Psi/(2 a^2 c^2))
    Phi = xi / chi                           # xi = Phi (1 - Psi/(2 a^2 c^2))
    alpha = 1 + Phi / (a * a * c * c)
    X = (x, y, z)
    src = [2 * a ** 3 * sum(sp.diff(alpha * psi ** -6 * A[(i, j)], X[j]) for j in range(3)) for i in range(3)]
    lam = lambda e: sp.lambdify(X, e, "numpy")
    fields = dict(Psi=lam(Psi), xi=lam(xi), A6=[lam(A[k]) for k in ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))])
    return [lam(e) for e in src], fields


def _eval(fn, X, Y, Z):
    return np.broadcast_to(np.asarray(fn(X, Y, Z), dtype=np.float64), X.shape).copy()


@pytest.mark.parametrize("a,c", [(0.6, 1.1), (1.3, 0.8)])
def test_shift_source_converges_to_continuum_md_equation(a, c):
    """Periodic oracle: error against the continuum MD-gauge source falls by
    4 +- 0.4 from 32^3 to 64^3 (and chi spans well beyond 1 +- 0.2, so a wrong
    chi power, a missing 1/chi in Phi or a stray a^3 fails at order one)."""
    src, F = _shift_source_continuum(a, c)
    prm = O.params(a=a, omega_m=0.3, c_tilde=c)
    errs = []
    for n in (32, 64):
        X, Y, Z = centres(n)
        psi, xi = _eval(F["Psi"], X, Y, Z), _eval(F["xi"], X, Y, Z)
        chi = 1 - psi / (2 * a * a * c * c)
        assert chi.min() < 0.6 and chi.max() > 1.4
        A6 = np.stack([_eval(f, X, Y, Z) for f in F["A6"]])
        out = O.build_shift_source(psi, xi, A6, prm=prm)
        ref = [_eval(f, X, Y, Z) for f in src]
        errs.append(max(maxrel(out[i], ref[i]) for i in range(3)))
    assert errs[0] < 0.2
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_patch_shift_source_converges_to_continuum_md_equation():
    """Patch oracle: a patch of n^3 cells of spacing 1/(2n) anywhere in the
    box, padded fields sampled at the shell's cell centres; second order."""
    a, c = 0.6, 1.1
    src, F = _shift_source_continuum(a, c)
    prm = O.params(a=a, omega_m=0.3, c_tilde=c)
    errs = []
    for n in (24, 48):
        h = 0.5 / n
        g = 0.3 + (np.arange(-1, n + 1) + 0.5) * h           # padded cell centres
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        psi, xi = _eval(F["Psi"], X, Y, Z), _eval(F["xi"], X, Y, Z)
        A6 = np.stack([_eval(f, X, Y, Z) for f in F["A6"]])
        out = D.build_shift_source(psi, xi, A6, h, prm)
        sl = (slice(1, -1),) * 3
        ref = [_eval(f, X[sl], Y[sl], Z[sl]) for f in src]
        errs.append(max(maxrel(out[i], ref[i]) for i in range(3)))
    assert errs[0] < 0.2
    assert 3.6 < errs[0] / errs[1] < 4.4
