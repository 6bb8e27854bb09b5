"""Pins of the Dirichlet-patch oracle (oracle/dirichlet.py) against what the
mathematics fixes: dense linear solves on tiny grids, manufactured solutions
of the code-unit Hamiltonian constraint (sec. 4.1.1), second-order convergence
to a continuum solution, the V-cycle factor, scipy's linear interpolation, and
the periodic oracle's source builders on an aligned copy of a parent region.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from oracle import dirichlet as D
from paper_1905_08890_amd import synth

STRESS = O.params(a=1.0, omega_m=0.3072, c_tilde=1.0)   # kappa = 1/2: strongly nonlinear


def maxrel(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def padded_random(rng, n, scale=1.0):
    return scale * rng.standard_normal((n + 2, n + 2, n + 2))


def dense_dirichlet(n, h, bnd, f, m2=None):
    """Brute force: the 7-point operator Lap - m2 on the n^3 interior as a
    dense matrix, where the value across a boundary face is 2 b - phi_cell
    (b in the padded array's face cells): -1/h^2 more on the diagonal per
    boundary face and 2 b/h^2 moved to the right-hand side."""
    N = n ** 3
    A = np.zeros((N, N))
    b = np.array(f, dtype=np.float64).reshape(-1).copy()
    idx = lambda i, j, k: (k * n + j) * n + i
    for k in range(n):
        for j in range(n):
            for i in range(n):
                r = idx(i, j, k)
                A[r, r] = -6.0 / h ** 2 - (0.0 if m2 is None else m2[k, j, i])
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < n and 0 <= jj < n and 0 <= kk < n:
                        A[r, idx(ii, jj, kk)] += 1.0 / h ** 2
                    else:
                        A[r, r] -= 1.0 / h ** 2
                        b[r] -= 2.0 * bnd[kk + 1, jj + 1, ii + 1] / h ** 2
    return np.linalg.solve(A, b).reshape(n, n, n)


def test_levels_follow_the_halving_rule():
    coarsest = {24: 3, 32: 4, 40: 5, 48: 3, 56: 7, 64: 4, 72: 9, 80: 5}
    for n, c in coarsest.items():
        s = D.levels(n)
        assert s[0] == n and s[-1] == c
        assert all(a == 2 * b for a, b in zip(s, s[1:]))


@pytest.mark.parametrize("n", [6, 8, 12])
def test_poisson_matches_dense_solve(n):
    """Random source and random boundary values on every level: the converged
    solve is the dense solution, whatever the coarse levels' boundary values
    are (FAS consistency)."""
    rng = np.random.default_rng(n)
    h = 1.0 / n
    g0 = padded_random(rng, n)
    f = rng.standard_normal((n, n, n))
    coarse = [padded_random(rng, m) for m in D.levels(n)[1:]]
    phi = g0.copy()
    D.interior(phi)[...] = 0.0
    out, st, cyc, rel = D.solve(D.POISSON, phi, f, None, coarse, h, STRESS, rtol=1e-13, max_cycles=60)
    assert st == D.OK
    ref = dense_dirichlet(n, h, g0, f)
    assert maxrel(D.interior(out), ref) < 1e-12
    # the padding (boundary values) is left as given
    shell = np.ones_like(g0, dtype=bool)
    D.interior(shell)[...] = False
    assert np.array_equal(out[shell], g0[shell])


def test_cmc_matches_dense_solve():
    n = 8
    rng = np.random.default_rng(3)
    h = 1.0 / n
    g0 = padded_random(rng, n)
    f = rng.standard_normal((n, n, n))
    m2 = 50.0 * rng.random((n, n, n))
    coarse = [padded_random(rng, m) for m in D.levels(n)[1:]]
    phi = g0.copy()
    D.interior(phi)[...] = 0.0
    out, st, cyc, rel = D.solve(D.CMC, phi, f, m2, coarse, h, STRESS, rtol=1e-13, max_cycles=60)
    assert st == D.OK
    assert maxrel(D.interior(out), dense_dirichlet(n, h, g0, f, m2)) < 1e-12


def face_lap(psi, bnd, h):
    """Discrete Laplacian of interior values psi (n^3) with face values bnd
    (padded): across a boundary face the neighbour is 2 b - psi_cell."""
    n = psi.shape[0]
    p = np.zeros((n + 2,) * 3)
    p[1:-1, 1:-1, 1:-1] = psi
    p[0, 1:-1, 1:-1] = 2 * bnd[0, 1:-1, 1:-1] - psi[0]
    p[-1, 1:-1, 1:-1] = 2 * bnd[-1, 1:-1, 1:-1] - psi[-1]
    p[1:-1, 0, 1:-1] = 2 * bnd[1:-1, 0, 1:-1] - psi[:, 0]
    p[1:-1, -1, 1:-1] = 2 * bnd[1:-1, -1, 1:-1] - psi[:, -1]
    p[1:-1, 1:-1, 0] = 2 * bnd[1:-1, 1:-1, 0] - psi[:, :, 0]
    p[1:-1, 1:-1, -1] = 2 * bnd[1:-1, 1:-1, -1] - psi[:, :, -1]
    return (p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] + p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1]
            + p[2:, 1:-1, 1:-1] + p[:-2, 1:-1, 1:-1] - 6.0 * psi) / h ** 2


def hamiltonian_f(psi, bnd, AA, h, prm):
    """f = 3/2 a Om (s0 - 1) with s0 from the code-unit Hamiltonian constraint
    chi Lap Psi = 3/2 a Om [s0 - chi^6] + AA/4 chi^-6 (discrete Laplacian with
    face values)."""
    kap = 1.0 / (2.0 * prm.a ** 2 * prm.c_tilde ** 2)
    A = 1.5 * prm.a * prm.omega_m
    lap = face_lap(psi, bnd, h)
    chi = 1.0 - kap * psi
    s0 = chi ** 6 + (chi * lap - 0.25 * AA * chi ** -6) / A
    return A * (s0 - 1.0)


@pytest.mark.parametrize("n", [12, 16])
def test_hamiltonian_manufactured_discrete(n):
    """A smooth Psi* (chi* in [0.6, 1.4] at the stress parameters), random
    face values, AA >= 0, s0 made from them by the constraint: the solve
    returns Psi* to rounding."""
    rng = np.random.default_rng(10 + n)
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    psi = 0.6 * np.sin(2.3 * X + 0.4) * np.cos(1.7 * Y - 0.2) * np.sin(2.9 * Z + 1.0) + 0.05
    bnd = padded_random(rng, n, 0.3)
    AA = 30.0 * rng.random((n, n, n))
    f = hamiltonian_f(psi, bnd, AA, h, STRESS)
    phi = bnd.copy()
    D.interior(phi)[...] = 0.0
    coarse = [padded_random(rng, m, 0.1) for m in D.levels(n)[1:]]
    out, st, cyc, rel = D.solve(D.HAMILTONIAN, phi, f, AA, coarse, h, STRESS, rtol=1e-14, max_cycles=80)
    assert st == D.OK
    assert maxrel(D.interior(out), psi) < 1e-12


def test_poisson_second_order_against_continuum():
    """phi = cos(x) e^{y} sin(z + 1/2) + x y z^2 (not zero anywhere on the
    boundary) on the unit cube, with its values at the face centres as the
    boundary values on every level: the error falls ~4x per halving of h."""
    def exact(X, Y, Z):
        return np.cos(X) * np.exp(Y) * np.sin(Z + 0.5) + X * Y * Z ** 2

    def lap_exact(X, Y, Z):
        return -np.cos(X) * np.exp(Y) * np.sin(Z + 0.5) + 2.0 * X * Y

    def faces(m):
        hm = 1.0 / m
        u = np.concatenate(([0.0], (np.arange(m) + 0.5) * hm, [1.0]))
        Z, Y, X = np.meshgrid(u, u, u, indexing="ij")
        b = np.zeros((m + 2,) * 3)
        I = slice(1, m + 1)
        for sl in ((0, I, I), (m + 1, I, I), (I, 0, I), (I, m + 1, I), (I, I, 0), (I, I, m + 1)):
            b[sl] = exact(X, Y, Z)[sl]
        return b

    errs = []
    for n in (16, 32):
        h = 1.0 / n
        x = (np.arange(n) + 0.5) * h
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        phi = faces(n)
        out, st, cyc, rel = D.solve(D.POISSON, phi, lap_exact(X, Y, Z), None,
                                    [faces(m) for m in D.levels(n)[1:]], h, STRESS, rtol=1e-12)
        assert st == D.OK
        errs.append(np.max(np.abs(D.interior(out) - exact(X, Y, Z))))
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.mark.parametrize("kind", [D.POISSON, D.HAMILTONIAN, D.CMC])
def test_vcycle_convergence_factor(kind):
    """Asymptotic residual reduction per V(2,2) cycle below 0.2 (48 -> 3)."""
    n = 48
    rng = np.random.default_rng(5)
    h = 1.0 / n
    prm = O.params()
    g0 = padded_random(rng, n, 1e-3)
    f = synth.grf(n, 4, -2.0, 1.0)
    coef = None if kind == D.POISSON else 100.0 * rng.random((n, n, n))
    coarse = [padded_random(rng, m, 1e-3) for m in D.levels(n)[1:]]
    phi = g0.copy()
    D.interior(phi)[...] = 0.0
    rels = []
    for k in range(1, 7):
        _, st, cyc, rel = D.solve(kind, phi, f, coef, coarse, h, prm, rtol=0.0, max_cycles=k)
        rels.append(rel)
    factor = (rels[-1] / rels[-3]) ** 0.5
    assert factor < 0.2


def test_face_values_are_parent_samples_at_face_centres():
    """Face cells of the padding hold the parent interpolated at the face
    centres (scipy, order 1, grid-wrap); edges, corners and interior are 0."""
    rng = np.random.default_rng(4)
    N, H = 10, 0.1
    parent = rng.standard_normal((N, N, N))
    n, h, origin = 6, H / 2, (0.7, 0.15, 0.95)
    out = D.face_values(parent, H, n, h, origin)
    u = np.concatenate(([0.0], np.arange(n) + 0.5, [float(n)]))
    c = [(o + u * h) / H - 0.5 for o in origin]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    ref = ndimage.map_coordinates(parent, [Z.ravel(), Y.ravel(), X.ravel()], order=1,
                                  mode="grid-wrap").reshape(out.shape)
    face = np.zeros(out.shape, dtype=bool)
    I = slice(1, n + 1)
    for sl in ((0, I, I), (n + 1, I, I), (I, 0, I), (I, n + 1, I), (I, I, 0), (I, I, n + 1)):
        face[sl] = True
    assert np.max(np.abs(out[face] - ref[face])) < 1e-13
    assert np.all(out[~face] == 0.0)


def test_sample_parent_matches_scipy_linear_interpolation():
    """The ghost sampler is linear interpolation at cell-centred coordinates,
    periodic in the parent: scipy's map_coordinates (order 1, grid-wrap)."""
    rng = np.random.default_rng(1)
    N, H = 12, 1.0 / 12
    parent = rng.standard_normal((N, N, N))
    for n, h, origin in ((6, H / 2, (3 * H, 0.0, 9 * H)), (8, H / 2, (10 * H, 5 * H, 11 * H)),
                         (5, H / 3, (0.37, 0.81, 0.05))):
        out = D.sample_parent(parent, H, n, h, origin)
        c = [(o + (np.arange(-1, n + 1) + 0.5) * h) / H - 0.5 for o in origin]
        Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
        ref = ndimage.map_coordinates(parent, [Z.ravel(), Y.ravel(), X.ravel()], order=1,
                                      mode="grid-wrap").reshape(out.shape)
        assert np.max(np.abs(out - ref)) < 1e-13


def test_sample_parent_exact_on_linear_fields():
    N, H = 16, 1.0 / 16
    x = (np.arange(N) + 0.5) * H
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    parent = 0.3 + 1.1 * X - 0.7 * Y + 2.0 * Z
    n, h, origin = 8, H / 2, (4 * H, 5 * H, 3 * H)       # well inside: no wrap
    out = D.sample_parent(parent, H, n, h, origin)
    c = [o + (np.arange(-1, n + 1) + 0.5) * h for o in origin]
    z, y, xx = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    assert np.max(np.abs(out - (0.3 + 1.1 * xx - 0.7 * y + 2.0 * z))) < 1e-13


def test_patch_builders_match_periodic_builders_on_aligned_copy():
    """A patch at the parent's own spacing, aligned with its cells, samples the
    parent exactly; its source builders must then equal the periodic oracle's
    builders on that region (A_ij, A_ij A^ij, -1/4 d.V, the shift source)."""
    N = 16
    H = 1.0 / N
    prm = O.params()
    rng = np.random.default_rng(2)
    F = {k: synth.grf(N, 20 + i, -3.0, 1e-3) for i, k in enumerate(O.FIELDS)}
    A6, AA = O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])
    fU = O.build_div_quarter(F["Vx"], F["Vy"], F["Vz"])
    fB = O.build_shift_source(F["Psi"], F["xi"], A6, prm)
    n, off = 8, (5, 11, 3)                                  # wraps in y
    origin = tuple(o * H for o in off)
    sl = np.ix_(*[np.arange(off[a], off[a] + n) % N for a in (2, 1, 0)])
    P = {k: D.sample_parent(F[k], H, n, H, origin) for k in O.FIELDS}
    assert np.array_equal(D.interior(P["U"]), F["U"][sl])
    pA6, pAA = D.build_Aij([P["Vx"], P["Vy"], P["Vz"]], P["U"], H)
    assert maxrel(pAA, AA[sl]) < 1e-13
    for c in range(6):
        assert maxrel(pA6[c], A6[c][sl]) < 1e-13
    assert maxrel(D.div_quarter(P["Vx"], P["Vy"], P["Vz"], H), fU[sl]) < 1e-13
    A6p = np.stack([D.sample_parent(A6[c], H, n, H, origin) for c in range(6)])
    pB = D.build_shift_source(P["Psi"], P["xi"], A6p, H, prm)
    for d in range(3):
        assert maxrel(pB[d], fB[d][sl]) < 1e-12
    m2, f = O.build_cmc(F["Psi"], 1.0 + F["U"], F["b"], AA, prm)
    pm2, pf = D.build_cmc(D.interior(P["Psi"]), 1.0 + D.interior(P["U"]), D.interior(P["b"]), pAA, prm)
    assert maxrel(pm2, m2[sl]) < 1e-13 and maxrel(pf, f[sl]) < 1e-13


def test_patch_of_a_solved_parent_at_same_spacing_reproduces_it():
    """Whole-patch pin: a parent solved by the periodic oracle with momentum
    sources of zero mean and a patch that copies a region of it at the same
    spacing.  Patch and parent solve the same discrete equations there except
    for the parent's regularisation constants <F> and <f> + <m^2 xi>, so the
    Poisson-kind fields V_i, U, B^i, b must be reproduced to the solve
    tolerance; Psi and xi may differ by the regularisation only (checked
    loosely)."""
    N = 16
    H = 1.0 / N
    prm = O.params()
    s0 = 1.0 + synth.grf(N, 31, -2.0, 0.1)
    sx, sy, sz = (synth.grf(N, 32 + d, -3.0, 1e-3) for d in range(3))
    sm = np.zeros((N, N, N))
    F, st, cyc, rel, AAp = O.solve_all(s0, sx, sy, sz, sm, rtol=1e-13)
    assert st == O.OK
    A6, _ = O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])
    n, off = 8, (3, 14, 6)
    origin = tuple(o * H for o in off)
    sl = np.ix_(*[np.arange(off[a], off[a] + n) % N for a in (2, 1, 0)])
    src = dict(s0=s0[sl], sx=sx[sl], sy=sy[sl], sz=sz[sl], sm=sm[sl])
    out, pst, pcyc, prel, pAA = D.solve_patch(F, A6, H, src, n, H, origin, prm, rtol=1e-13)
    assert pst == D.OK
    for k in ("Vx", "Vy", "Vz", "U", "Bx", "By", "Bz", "b"):
        assert maxrel(D.interior(out[k]), F[k][sl]) < 1e-9, k
    for k in ("Psi", "xi"):
        assert maxrel(D.interior(out[k]), F[k][sl]) < 5e-2, k


def test_nested_sampling_matches_scipy_inside_and_refuses_outside():
    """A parent patch is sampled without wrap (reading D6): scipy's linear
    interpolation (order 1) at interior points, exact on linear fields, and a
    child too close to the parent's faces is refused."""
    rng = np.random.default_rng(7)
    N, H = 12, 1.0 / 24
    parent = rng.standard_normal((N, N, N))
    n, h = 8, H / 2
    origin = (1.5 * H, 2.0 * H, 3.0 * H)          # >= (H + h)/2 inside every face
    out = D.sample_parent(parent, H, n, h, origin, periodic=False)
    c = [(o + (np.arange(-1, n + 1) + 0.5) * h) / H - 0.5 for o in origin]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    ref = ndimage.map_coordinates(parent, [Z.ravel(), Y.ravel(), X.ravel()], order=1).reshape(out.shape)
    assert np.max(np.abs(out - ref)) < 1e-13
    fv = D.face_values(parent, H, n, h, origin, periodic=False)
    u = np.concatenate(([0.0], np.arange(n) + 0.5, [float(n)]))
    c = [(o + u * h) / H - 0.5 for o in origin]
    Z, Y, X = np.meshgrid(c[2], c[1], c[0], indexing="ij")
    ref = ndimage.map_coordinates(parent, [Z.ravel(), Y.ravel(), X.ravel()], order=1).reshape(fv.shape)
    I = slice(1, n + 1)
    for sl in ((0, I, I), (n + 1, I, I), (I, 0, I), (I, n + 1, I), (I, I, 0), (I, I, n + 1)):
        assert np.max(np.abs(fv[sl] - ref[sl])) < 1e-13
    x = (np.arange(N) + 0.5) * H
    Zp, Yp, Xp = np.meshgrid(x, x, x, indexing="ij")
    lin_f = 0.2 - 0.9 * Xp + 1.3 * Yp + 0.4 * Zp
    got = D.sample_parent(lin_f, H, n, h, origin, periodic=False)
    cc = [o + (np.arange(-1, n + 1) + 0.5) * h for o in origin]
    z, y, xx = np.meshgrid(cc[2], cc[1], cc[0], indexing="ij")
    assert np.max(np.abs(got - (0.2 - 0.9 * xx + 1.3 * y + 0.4 * z))) < 1e-13
    for bad in ((0.5 * H, 2.0 * H, 3.0 * H), (1.5 * H, 2.0 * H, (N - 4.5) * H)):
        with pytest.raises(ValueError):
            D.sample_parent(parent, H, n, h, bad, periodic=False)


def test_nested_patch_at_same_spacing_reproduces_its_parent_patch():
    """Nested pin: a patch (the first refinement of a solved periodic box)
    and, inside it, a child patch at the same spacing aligned with its cells
    and fed the same sources.  Both solve the plain discrete equations (no
    regularisation on patches), and the child's face values and outside
    stencil values are the parent patch's own cells, so all ten fields of the
    child equal the parent patch's on that block to the solve tolerance."""
    N = 16
    H = 1.0 / N
    prm = O.params()
    s0 = 1.0 + synth.grf(N, 41, -2.0, 0.1)
    sx, sy, sz = (synth.grf(N, 42 + d, -3.0, 1e-3) for d in range(3))
    sm = np.zeros((N, N, N))
    F, st, *_ = O.solve_all(s0, sx, sy, sz, sm, rtol=1e-13)
    assert st == O.OK
    A6, _ = O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])
    # level 1: 12^3 at H/2, lower corner at parent cell (3, 5, 2)
    n1, h1, o1 = 12, H / 2, (3 * H, 5 * H, 2 * H)
    rng = np.random.default_rng(9)
    src1 = dict(s0=1.0 + 0.1 * rng.standard_normal((n1,) * 3), sm=np.zeros((n1,) * 3),
                **{k: 1e-3 * rng.standard_normal((n1,) * 3) for k in ("sx", "sy", "sz")})
    P1, st1, c1, r1, AA1, A61 = D.solve_patch(F, A6, H, src1, n1, h1, o1, prm, rtol=1e-13, return_A6=True)
    assert st1 == D.OK
    # level 2: 6^3 at the same spacing, 3 cells inside the parent patch
    n2, off = 6, (3, 2, 4)
    o2 = tuple(k * h1 for k in off)
    sl = np.ix_(*[np.arange(off[a], off[a] + n2) for a in (2, 1, 0)])
    src2 = {k: v[sl] for k, v in src1.items()}
    parent = {k: D.interior(P1[k]) for k in D.FIELDS}
    P2, st2, *_ = D.solve_patch(parent, A61, h1, src2, n2, h1, o2, prm, rtol=1e-13, periodic=False)
    assert st2 == D.OK
    for k in D.FIELDS:
        assert maxrel(D.interior(P2[k]), parent[k][sl]) < 1e-9, k
