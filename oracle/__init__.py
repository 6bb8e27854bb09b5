"""ctypes shim over the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  The oracle and
the GPU library share no code; both only consume the same seeded inputs.

Every function takes and returns C-contiguous float64 numpy arrays laid out
[z][y][x] (x fastest) on a periodic n^3 box.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

POISSON, HAMILTONIAN, CMC = 0, 1, 2
FIELDS = ("Vx", "Vy", "Vz", "U", "Psi", "xi", "Bx", "By", "Bz", "b")
OK, EINVAL, ENOTCONV, ENAN, ENOMEM = 0, -1, -3, -4, -5


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("a", C.c_double), ("omega_m", C.c_double), ("c_tilde", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int), ("rtol", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER(C.c_double)
        _lib.orc_num_levels.argtypes = [C.c_int]
        _lib.orc_solve_equation.argtypes = [C.c_int, C.c_double, C.POINTER(_Params), C.c_int, P, P, P,
                                            C.POINTER(_Opts), C.POINTER(C.c_int), P]
        _lib.orc_rb_sweep.argtypes = [C.c_int, C.c_double, C.POINTER(_Params), C.c_int, C.c_double,
                                      C.c_double, P, P, P]
        _lib.orc_residual.argtypes = [C.c_int, C.c_double, C.POINTER(_Params), C.c_int, C.c_double,
                                      C.c_double, P, P, P, P]
        _lib.orc_restrict.argtypes = [C.c_int, P, P]
        _lib.orc_prolong_add.argtypes = [C.c_int, P, P]
        _lib.orc_interp_cubic.argtypes = [C.c_int, P, P]
        _lib.orc_cic_deposit.argtypes = [C.c_int, C.POINTER(_Params), C.c_long, P, P, C.c_double, P,
                                         P, P, P, P, P]
        _lib.orc_build_Aij.argtypes = [C.c_int, P, P, P, P, P, P]
        _lib.orc_build_div_quarter.argtypes = [C.c_int, P, P, P, P]
        _lib.orc_build_cmc.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, P]
        _lib.orc_build_shift_source.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, P]
        _lib.orc_solve_all.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, C.POINTER(P),
                                       C.c_int, C.c_int, C.POINTER(C.c_int), C.c_double,
                                       C.POINTER(C.c_int), P, P]
        _lib.orc_derived.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, P, P, P, P, P]
        _lib.orc_cycle_residual.argtypes = [C.c_int, C.c_double, C.POINTER(_Params), C.c_int, P, P, P]
        _lib.orc_cycle_residual.restype = C.c_double
        _lib.orc_kick.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, C.c_long, P, P, C.c_double, C.c_int]
        _lib.orc_drift.argtypes = [C.c_int, C.POINTER(_Params), P, P, P, P, P, C.c_long, P, P, C.c_double]
        _lib.orc_newtonian_kick.argtypes = [C.c_int, C.POINTER(_Params), P, P, C.c_long, P, P, C.c_double,
                                            C.c_double, C.c_int, C.POINTER(C.c_int)]
    return _lib


def _p(x: np.ndarray):
    assert x.dtype == np.float64 and x.flags.c_contiguous
    return x.ctypes.data_as(C.POINTER(C.c_double))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def params(a=1.0, omega_m=0.3072, c_tilde=2997.92458 / 256.0) -> _Params:
    return _Params(a, omega_m, c_tilde)


def num_levels(n: int) -> int:
    return lib().orc_num_levels(n)


def solve_equation(kind, phi, f, coef=None, prm=None, h=None, nu1=2, nu2=2, max_cycles=100,
                   rtol=1e-10):
    """Solve one equation; returns (phi, status, cycles, rel_residual)."""
    prm = prm or params()
    phi = _f64(phi).copy()
    f = _f64(f)
    n = phi.shape[0]
    coef = _f64(coef) if coef is not None else np.zeros_like(phi)
    cyc, rel = C.c_int(0), C.c_double(0.0)
    o = _Opts(nu1, nu2, max_cycles, rtol)
    st = lib().orc_solve_equation(n, h if h is not None else 1.0 / n, C.byref(prm), kind, _p(phi),
                                  _p(f), _p(coef), C.byref(o), C.byref(cyc), C.byref(rel))
    return phi, st, cyc.value, rel.value


def rb_sweep(kind, phi, f, coef=None, prm=None, h=None, Fbar=0.0, fshift=0.0):
    prm = prm or params()
    phi = _f64(phi).copy()
    coef = _f64(coef) if coef is not None else np.zeros_like(phi)
    n = phi.shape[0]
    lib().orc_rb_sweep(n, h if h is not None else 1.0 / n, C.byref(prm), kind, Fbar, fshift, _p(phi),
                       _p(_f64(f)), _p(coef))
    return phi


def residual(kind, phi, f, coef=None, prm=None, h=None, Fbar=0.0, fshift=0.0):
    prm = prm or params()
    phi = _f64(phi)
    coef = _f64(coef) if coef is not None else np.zeros_like(phi)
    r = np.empty_like(phi)
    n = phi.shape[0]
    lib().orc_residual(n, h if h is not None else 1.0 / n, C.byref(prm), kind, Fbar, fshift, _p(phi),
                       _p(_f64(f)), _p(coef), _p(r))
    return r


def restrict(fine):
    fine = _f64(fine)
    n = fine.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().orc_restrict(n, _p(fine), _p(out))
    return out


def prolong_add(e, fine):
    e = _f64(e)
    fine = _f64(fine).copy()
    lib().orc_prolong_add(e.shape[0], _p(e), _p(fine))
    return fine


def interp_cubic(coarse):
    """Cubic (Lagrange, 4 points per dimension) interpolation of a coarse m^3
    field to (2m)^3 cell centres (periodic)."""
    coarse = _f64(coarse)
    m = coarse.shape[0]
    out = np.empty((2 * m,) * 3)
    lib().orc_interp_cubic(m, _p(coarse), _p(out))
    return out


def cic_deposit(n, pos, u, mass, psi=None, prm=None):
    """Returns (s0, sx, sy, sz, sm)."""
    prm = prm or params()
    pos = _f64(pos).reshape(-1, 3)
    u = _f64(u).reshape(-1, 3)
    outs = [np.empty((n, n, n)) for _ in range(5)]
    psi_p = _p(_f64(psi)) if psi is not None else None
    lib().orc_cic_deposit(n, C.byref(prm), pos.shape[0], _p(pos), _p(u), mass, psi_p,
                          *[_p(o) for o in outs])
    return tuple(outs)


def build_Aij(Vx, Vy, Vz, U):
    """Returns (Aij[6] packed xx,yy,zz,xy,xz,yz ; AA)."""
    n = U.shape[0]
    A6 = np.empty((6, n, n, n))
    AA = np.empty((n, n, n))
    lib().orc_build_Aij(n, _p(_f64(Vx)), _p(_f64(Vy)), _p(_f64(Vz)), _p(_f64(U)), _p(A6), _p(AA))
    return A6, AA


def build_div_quarter(gx, gy, gz):
    n = gx.shape[0]
    f = np.empty((n, n, n))
    lib().orc_build_div_quarter(n, _p(_f64(gx)), _p(_f64(gy)), _p(_f64(gz)), _p(f))
    return f


def build_cmc(psi, s0, sm, AA, prm=None):
    prm = prm or params()
    n = psi.shape[0]
    m2 = np.empty((n, n, n))
    f = np.empty((n, n, n))
    lib().orc_build_cmc(n, C.byref(prm), _p(_f64(psi)), _p(_f64(s0)), _p(_f64(sm)), _p(_f64(AA)),
                        _p(m2), _p(f))
    return m2, f


def build_shift_source(psi, xi, A6, prm=None):
    prm = prm or params()
    n = psi.shape[0]
    outs = [np.empty((n, n, n)) for _ in range(3)]
    lib().orc_build_shift_source(n, C.byref(prm), _p(_f64(psi)), _p(_f64(xi)), _p(_f64(A6)),
                                 *[_p(o) for o in outs])
    return tuple(outs)


def solve_all(s0, sx, sy, sz, sm, guesses=None, prm=None, nu1=2, nu2=2, max_cycles=100,
              rtol=1e-10):
    """Solve all ten fields.  Returns (dict field->array, status, cycles[10], rel[10], AA)."""
    prm = prm or params()
    n = s0.shape[0]
    fields = [(_f64(guesses[k]).copy() if guesses is not None and k in guesses else np.zeros((n, n, n)))
              for k in FIELDS]
    ptrs = (C.POINTER(C.c_double) * 10)(*[_p(x) for x in fields])
    mc = np.broadcast_to(np.asarray(max_cycles, dtype=np.int32), (10,)).copy()
    cycles = (C.c_int * 10)()
    rel = (C.c_double * 10)()
    AA = np.empty((n, n, n))
    st = lib().orc_solve_all(n, C.byref(prm), _p(_f64(s0)), _p(_f64(sx)), _p(_f64(sy)), _p(_f64(sz)),
                             _p(_f64(sm)), ptrs, nu1, nu2, mc.ctypes.data_as(C.POINTER(C.c_int)), rtol,
                             cycles, rel, _p(AA))
    return dict(zip(FIELDS, fields)), st, list(cycles), list(rel), AA


def cycle_residual(kind, phi, f, coef=None, prm=None, h=None):
    """rms(eps)/rms(f) of a pinned iterate with the frozen means evaluated from it."""
    prm = prm or params()
    phi = _f64(phi)
    coef = _f64(coef) if coef is not None else np.zeros_like(phi)
    n = phi.shape[0]
    return lib().orc_cycle_residual(n, h if h is not None else 1.0 / n, C.byref(prm), kind, _p(phi),
                                    _p(_f64(f)), _p(coef))


def derived(psi, xi, Bx, By, Bz, b, prm=None):
    """Returns (Phi, beta_x, beta_y, beta_z)."""
    prm = prm or params()
    n = psi.shape[0]
    outs = [np.empty((n, n, n)) for _ in range(4)]
    lib().orc_derived(n, C.byref(prm), *[_p(_f64(x)) for x in (psi, xi, Bx, By, Bz, b)],
                      *[_p(o) for o in outs])
    return tuple(outs)


KICK_FORWARD, KICK_REVERSE = 0, 1


def kick(Phi, Psi, beta, pos, u, dt, order=KICK_FORWARD, prm=None):
    """One kick of length dt (five substeps, sec. 4.4); returns the new u [np][3]."""
    prm = prm or params()
    n = Psi.shape[0]
    pos = _f64(pos).reshape(-1, 3)
    out = _f64(u).reshape(-1, 3).copy()
    bx, by, bz = (_f64(b) for b in beta)
    lib().orc_kick(n, C.byref(prm), _p(_f64(Phi)), _p(_f64(Psi)), _p(bx), _p(by), _p(bz), pos.shape[0], _p(pos),
                   _p(out), dt, order)
    return out


def drift(Phi, Psi, beta, pos, u, dt, prm=None):
    """Drift of length dt (sec. 4.4); returns the new positions [np][3] in [0, 1)."""
    prm = prm or params()
    n = Psi.shape[0]
    out = _f64(pos).reshape(-1, 3).copy()
    u = _f64(u).reshape(-1, 3)
    bx, by, bz = (_f64(b) for b in beta)
    lib().orc_drift(n, C.byref(prm), _p(_f64(Phi)), _p(_f64(Psi)), _p(bx), _p(by), _p(bz), out.shape[0], _p(out),
                    _p(u), dt)
    return out


def newtonian_kick(s0, pos, u, dt, prm=None, rtol=1e-10, max_cycles=100):
    """Newtonian potential Lap Phi_N = 3/2 a Om (s0 - 1) and the kick
    u -= dt grad Phi_N at the particles.  Returns (u_new, Phi_N, status, cycles)."""
    prm = prm or params()
    n = s0.shape[0]
    pos = _f64(pos).reshape(-1, 3)
    out = _f64(u).reshape(-1, 3).copy()
    phiN = np.empty((n, n, n))
    cyc = C.c_int()
    st = lib().orc_newtonian_kick(n, C.byref(prm), _p(_f64(s0)), _p(phiN), pos.shape[0], _p(pos), _p(out), dt,
                                  rtol, max_cycles, C.byref(cyc))
    return out, phiN, st, cyc.value
