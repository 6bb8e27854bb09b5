"""Pins of the oracle's particle evolution (kick and drift, sec. 4.4 and the
appendix on the leapfrog scheme) against what the paper fixes independently
of the printed force formula.

* Hamilton's equations: the appendix derives the geodesic equations from the
  3+1 Hamiltonian of a free particle, H = alpha sqrt(m^2 + gamma^ij p_i p_j)
  - beta^i p_i with gamma^ij = psi^-4 delta^ij.  Written for the code-unit
  momenta u and time of sec. 4.4 (H/m scaled by a^2 c, so that dH/du is the
  printed dx/dt), H = a^2 c alpha W - beta.u with W = sqrt(c^2 + psi^-4 u.u),
  psi = a^(1/2) (1 - Psi/(2a^2c^2)), alpha = 1 + Phi/(a^2c^2).  Its
  derivatives are taken symbolically for smooth, strongly relativistic fields
  (|u| ~ c, chi and alpha far from 1); the oracle's kick (du/dt from a tiny
  step, both substep orders) must converge to -dH/dx and its drift to dH/du
  at second order in the grid spacing.
* The substep order changes the kick only at second order in dt.
* FLRW: with all fields zero a kick leaves u unchanged and a drift moves a
  particle by dt c u / W exactly.
"""
import numpy as np
import pytest
import sympy as sp

import oracle as O
from closed_forms import centres

A, CT = 0.8, 1.5
PRM = O.params(a=A, omega_m=0.3072, c_tilde=CT)


def _continuum():
    x, y, z = sp.symbols("x y z", real=True)
    u = sp.symbols("u0:3", real=True)
    tp = 2 * sp.pi
    a, c = sp.Rational(4, 5), sp.Rational(3, 2)
    Phi = 0.35 * a * a * c * c * (sp.sin(tp * x) * sp.cos(tp * y) + 0.5 * sp.cos(tp * z + 0.4))
    Psi = 0.6 * a * a * c * c * (sp.cos(tp * x + 0.3) * sp.sin(tp * z) + 0.4 * sp.sin(tp * y))
    beta = [0.2 * sp.sin(tp * (y + z)), 0.15 * sp.cos(tp * x) * sp.sin(tp * z), 0.1 * sp.sin(tp * (x - y) + 0.7)]
    psi = sp.sqrt(a) * (1 - Psi / (2 * a * a * c * c))
    alpha = 1 + Phi / (a * a * c * c)
    uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    W = sp.sqrt(c * c + psi ** -4 * uu)
    H = a * a * c * alpha * W - sum(b * ui for b, ui in zip(beta, u))
    X = (x, y, z)
    args = X + tuple(u)
    lam = lambda e: sp.lambdify(args, e, "numpy")
    F = [lam(-sp.diff(H, X[i])) for i in range(3)]
    V = [lam(sp.diff(H, u[i])) for i in range(3)]
    grid = {k: sp.lambdify(X, e, "numpy") for k, e in (("Phi", Phi), ("Psi", Psi), ("bx", beta[0]),
                                                      ("by", beta[1]), ("bz", beta[2]))}
    return F, V, grid


@pytest.fixture(scope="module")
def cont():
    return _continuum()


def _fields(grid, n):
    X, Y, Z = centres(n)
    ev = lambda k: np.broadcast_to(np.asarray(grid[k](X, Y, Z), dtype=np.float64), X.shape).copy()
    return ev("Phi"), ev("Psi"), [ev("bx"), ev("by"), ev("bz")]


def _particles(npart=1000, seed=3):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.05, 0.95, (npart, 3))
    u = rng.uniform(-1.0, 1.0, (npart, 3)) * CT      # |u| ~ c: W^2 - c^2 of order c^2
    return pos, u


def test_kick_is_minus_dH_dx(cont):
    """du/dt of a tiny kick (both substep orders) converges to -dH/dx at
    second order: the rms error over 1000 random particles falls by 4 +- 0.4
    from 32^3 to 64^3 (the rms, not the maximum: the interpolation error of a
    particle depends on where it sits in its cell, which changes with n)."""
    F, _, grid = cont
    pos, u = _particles()
    ref = np.stack([f(*pos.T, *u.T) for f in F], axis=1)
    dt = 1e-7
    for order in (O.KICK_FORWARD, O.KICK_REVERSE):
        errs = []
        for n in (32, 64):
            Phi, Psi, beta = _fields(grid, n)
            un = O.kick(Phi, Psi, beta, pos, u, dt, order, prm=PRM)
            errs.append(np.sqrt((((un - u) / dt - ref) ** 2).mean()) / np.abs(ref).max())
        assert errs[0] < 0.01
        assert 3.6 < errs[0] / errs[1] < 4.4, (order, errs)


def test_drift_is_dH_du(cont):
    """dx/dt of a tiny drift converges to dH/du at second order (rms over the
    particles, as for the kick)."""
    _, V, grid = cont
    pos, u = _particles()
    ref = np.stack([v(*pos.T, *u.T) for v in V], axis=1)
    dt = 1e-7
    errs = []
    for n in (32, 64):
        Phi, Psi, beta = _fields(grid, n)
        xn = O.drift(Phi, Psi, beta, pos, u, dt, prm=PRM)
        d = (xn - pos + 0.5) % 1.0 - 0.5                 # minimal image
        errs.append(np.sqrt(((d / dt - ref) ** 2).mean()) / np.abs(ref).max())
    assert errs[0] < 0.01
    assert 3.6 < errs[0] / errs[1] < 4.4, errs


def test_substep_order_matters_at_second_order_in_dt(cont):
    """Forward and reverse substep orders differ by O(dt^2)."""
    _, _, grid = cont
    Phi, Psi, beta = _fields(grid, 32)
    pos, u = _particles(50, 5)
    diffs = []
    for dt in (2e-2, 1e-2):
        uf = O.kick(Phi, Psi, beta, pos, u, dt, O.KICK_FORWARD, prm=PRM)
        ur = O.kick(Phi, Psi, beta, pos, u, dt, O.KICK_REVERSE, prm=PRM)
        diffs.append(np.abs(uf - ur).max())
    assert diffs[0] > 0
    assert 3.6 < diffs[0] / diffs[1] < 4.4, diffs


def test_flrw_fields_leave_particles_on_straight_lines():
    """Zero fields (the homogeneous FLRW case): a kick changes nothing, a
    drift moves each particle by dt c u / W (W = sqrt(c^2 + u.u/a^2))."""
    n = 16
    z = np.zeros((n, n, n))
    pos, u = _particles(100, 7)
    for order in (O.KICK_FORWARD, O.KICK_REVERSE):
        assert np.array_equal(O.kick(z, z, [z, z, z], pos, u, 0.3, order, prm=PRM), u)
    dt = 1e-3
    W = np.sqrt(CT ** 2 + (u ** 2).sum(1) / A ** 2)
    ref = (pos + dt * CT * u / W[:, None]) % 1.0
    assert np.abs(O.drift(z, z, [z, z, z], pos, u, dt, prm=PRM) - ref).max() < 1e-15


def test_newtonian_potential_is_weak_field_psi():
    """The Newtonian potential of the temporary synchronisation solves the
    chi -> 1 limit of the Hamiltonian constraint, so for weak sources it
    equals the solved Psi up to the screening term mu^2 = 9 a Om kappa
    (relative 1e-3 at the default c~), and its kick on particles at rest is
    the GR kick's Newtonian term: u = -dt grad Psi there (rtol 1e-3)."""
    n = 32
    prm = O.params()
    s0 = 1.0 + 1e-3 * __import__("paper_1905_08890_amd.synth", fromlist=["grf"]).grf(n, 44, -2.0, 1.0)
    z = np.zeros((n, n, n))
    A_ = 1.5 * prm.a * prm.omega_m
    psi, st, _, _ = O.solve_equation(O.HAMILTONIAN, z, A_ * (s0 - 1.0), z, prm=prm, rtol=1e-13)
    pos, _ = _particles(300, 8)
    u0 = np.zeros_like(pos)
    uN, phiN, st2, cyc = O.newtonian_kick(s0, pos, u0, 0.1, prm=prm, rtol=1e-13)
    assert st == st2 == O.OK and cyc > 0
    assert np.abs(phiN - psi).max() < 1e-3 * np.abs(psi).max()
    assert abs(phiN.mean()) < 1e-14 * np.abs(phiN).max()
    uGR = O.kick(psi, z, [z, z, z], pos, u0, 0.1, O.KICK_FORWARD, prm=prm)   # Phi := Psi, no Psi, beta terms
    assert np.abs(uN - uGR).max() < 1e-3 * np.abs(uGR).max()
