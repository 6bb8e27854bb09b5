"""Dirichlet refinement patches: plain FP64 numpy oracle.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: imported by the tests and
the CPU-baseline leg of the benchmark, never by the product path.  It shares
no code with the GPU library.

A patch is a cube of n^3 cells of spacing h whose lower corner sits at
`origin` (box units) in the frame of its parent: a periodic box of N^3 cells
of spacing H, or (nested refinement) another patch of N^3 interior cells of
spacing H, whose frame starts at that patch's lower corner.  The iterate of every patch level is padded by one cell on each
side: shape (n+2, n+2, n+2), [z][y][x] with x fastest, interior [1:n+1]^3;
the cell across a face holds that face's boundary value (edge and corner
cells are zero and unused).  Sources, coefficients and right-hand sides are
interior arrays of shape (n, n, n).

The paper solves its refined levels with boundary values taken from the
coarser level (sec. 3, the AMR inherited from the parent code) and regularises
the periodic equations only because of the periodic boundary (sec. 4.3.1,
4.3.2.1, 4.3.2.2).  It prints no scheme for the refined levels, so these
readings are taken:
  D1 hierarchy: halve n while n is even and n/2 >= 3 (24, 32, 40, 48, 56,
     64, 72, 80 -> 3, 4, 5, 3, 7, 4, 9, 5); at the coarsest level 32
     red-black sweeps, with no mean projection.
  D2 boundary values on faces: on every level the boundary value b of a
     boundary face is the parent's solved field at the face centre, by
     cell-centred trilinear interpolation periodic in the parent.  The
     7-point stencil of a boundary cell takes across that face the linear
     extrapolation 2b - phi_cell (so the face average is b), and the Newton
     derivative counts it: -(6 + number of boundary faces)/h^2 in place of
     -6/h^2.  This places the boundary at the same faces on every level; with
     values at the ghost cell centres instead, the V-cycle factor grows with
     the depth (0.27 at 16^3, 0.63 at 48^3) because each coarse correction
     vanishes half a coarse cell further out than the fine error does.
  D3 no regularisation, no pin: the plain discrete equations (no <F>, <f> or
     <m^2 xi> terms, no mean removed from the momentum sources, no zero-mean
     pin).
  D4 FAS coarse equation on interior cells, f^H = L^H(R phi) - R eps with the
     coarse face values in the stencil; the correction phi^H - R phi is
     prolonged as an odd function across every face (zero on the face), so
     its value across a face is minus that of the adjacent cell.
  D5 sources as on the periodic box (sec. 4.3.1, 4.3.2.2); where a
     difference stencil reaches outside the patch it reads the parent's field
     (V_i, U, Psi, xi, B^i, b, and A_ij for d_j of the shift source) at that
     outside cell's centre, by the same interpolation.
  D6 nested refinement (the parent code's AMR hierarchy): a patch whose
     parent is a patch takes its boundary values and outside stencil values
     from that patch's solved interior by the same interpolation, without
     wrap; every sample must then fall strictly between the parent's cell
     centres (a child at least (H + h)/2 inside each face of its parent).
     Levels are solved coarse to fine, each with the finished field of the
     level above; the coarser levels' potentials are kept, so a refined level
     can be solved again (a sub-step) from them.
Red-black order, restriction (mean of 8 children), cell-centred trilinear
prolongation, Newton point update and the stopping test rms(eps)/rms(f) are
those of the periodic solver.
"""
from __future__ import annotations

import numpy as np

POISSON, HAMILTONIAN, CMC = 0, 1, 2
FIELDS = ("Vx", "Vy", "Vz", "U", "Psi", "xi", "Bx", "By", "Bz", "b")
OK, ENOTCONV, ENAN = 0, -3, -4
COARSE_SWEEPS = 32


def levels(n: int) -> list[int]:
    """Level sizes by reading D1."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= 3:
        sizes.append(sizes[-1] // 2)
    return sizes


def interior(a: np.ndarray) -> np.ndarray:
    return a[1:-1, 1:-1, 1:-1]


def _kappa(prm) -> float:
    return 1.0 / (2.0 * prm.a * prm.a * prm.c_tilde * prm.c_tilde)


# ----------------------------------------------------------------- ghosts

def _cells(g, N, periodic):
    """Per-axis cells and weight of the cell-centred linear interpolation at
    parent coordinates g (cell units, centres at integers): cells i0, i0 + 1
    with weights (1 - t, t).  Periodic: wrapped.  Non-periodic (a parent
    patch): every g must lie strictly inside (0, N - 1)."""
    i0 = np.floor(g)
    t = g - i0
    i0 = i0.astype(np.int64)
    if periodic:
        return np.mod(i0, N), np.mod(i0 + 1, N), t
    if np.any(g <= 0.0) or np.any(g >= N - 1):
        raise ValueError("nested patch too close to its parent's faces (reading D6)")
    return i0, i0 + 1, t


def sample_parent(parent: np.ndarray, H: float, n: int, h: float, origin, periodic: bool = True) -> np.ndarray:
    """Trilinear interpolation of a parent field (cell-centred, spacing H) at
    the (n+2)^3 cell centres origin + (i + 1/2) h, i = -1..n, of a padded
    patch level (reading D2).  Per axis: g = x/H - 1/2, i0 = floor(g),
    t = g - i0, weights (1 - t, t) on parent cells i0, i0 + 1 (wrapped for a
    periodic box; inside only for a parent patch, reading D6)."""
    N = parent.shape[0]
    idx = np.arange(-1, n + 1, dtype=np.float64)

    def axis(o):
        return _cells((o + (idx + 0.5) * h) / H - 0.5, N, periodic)

    x0, x1, tx = axis(origin[0])
    y0, y1, ty = axis(origin[1])
    z0, z1, tz = axis(origin[2])
    out = np.zeros((n + 2, n + 2, n + 2))
    for cz in (0, 1):
        wz = tz if cz else 1.0 - tz
        for cy in (0, 1):
            wy = ty if cy else 1.0 - ty
            for cx in (0, 1):
                wx = tx if cx else 1.0 - tx
                w = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                v = parent[np.ix_(z1 if cz else z0, y1 if cy else y0, x1 if cx else x0)]
                out += w * v
    return out


def face_values(parent: np.ndarray, H: float, n: int, h: float, origin, periodic: bool = True) -> np.ndarray:
    """Padded (n+2)^3 array whose cells across the six faces hold the parent
    sampled at the face centres (reading D2); everything else is zero."""
    N = parent.shape[0]
    u = np.concatenate(([0.0], np.arange(n) + 0.5, [float(n)]))    # face-clamped cell coordinates

    def axis(o):
        return _cells((o + u * h) / H - 0.5, N, periodic)

    x0, x1, tx = axis(origin[0])
    y0, y1, ty = axis(origin[1])
    z0, z1, tz = axis(origin[2])
    full = np.zeros((n + 2, n + 2, n + 2))
    for cz in (0, 1):
        wz = tz if cz else 1.0 - tz
        for cy in (0, 1):
            wy = ty if cy else 1.0 - ty
            for cx in (0, 1):
                wx = tx if cx else 1.0 - tx
                w = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
                full += w * parent[np.ix_(z1 if cz else z0, y1 if cy else y0, x1 if cx else x0)]
    out = np.zeros_like(full)
    for sl in _faces(n):
        out[sl] = full[sl]
    return out


def _faces(n):
    """Index expressions of the six face layers of the shell (no edges)."""
    I = slice(1, n + 1)
    return [(0, I, I), (n + 1, I, I), (I, 0, I), (I, n + 1, I), (I, I, 0), (I, I, n + 1)]


def boundary_of(parent: np.ndarray, H: float, n: int, h: float, origin, periodic: bool = True) -> list[np.ndarray]:
    """Face values of every level of the patch (reading D2)."""
    return [face_values(parent, H, m, h * (n // m), origin, periodic) for m in levels(n)]


# -------------------------------------------------------------- operators

def _nfaces(n: int) -> np.ndarray:
    """Number of boundary faces of every interior cell (0..3)."""
    a = np.zeros(n)
    a[0] += 1.0
    a[-1] += 1.0
    return a[:, None, None] + a[None, :, None] + a[None, None, :]


def lap(phi: np.ndarray, h: float):
    """7-point Laplacian at the interior of a padded array whose face cells
    hold boundary values b: across a face the stencil takes 2b - phi_cell
    (reading D2).  Returns the Laplacian and its derivative with respect to
    the cell's own value."""
    n = phi.shape[0] - 2
    c = interior(phi)
    nb = (phi[1:-1, 1:-1, :-2] + phi[1:-1, 1:-1, 2:] + phi[1:-1, :-2, 1:-1] + phi[1:-1, 2:, 1:-1]
          + phi[:-2, 1:-1, 1:-1] + phi[2:, 1:-1, 1:-1])
    # replace b by 2b - phi_cell on the boundary layers: add b - phi_cell once per face
    corr = np.zeros((n, n, n))
    corr[0, :, :] += phi[0, 1:-1, 1:-1] - c[0, :, :]
    corr[-1, :, :] += phi[-1, 1:-1, 1:-1] - c[-1, :, :]
    corr[:, 0, :] += phi[1:-1, 0, 1:-1] - c[:, 0, :]
    corr[:, -1, :] += phi[1:-1, -1, 1:-1] - c[:, -1, :]
    corr[:, :, 0] += phi[1:-1, 1:-1, 0] - c[:, :, 0]
    corr[:, :, -1] += phi[1:-1, 1:-1, -1] - c[:, :, -1]
    return (nb + corr - 6.0 * c) / (h * h), -(6.0 + _nfaces(n)) / (h * h)


def op(kind: int, phi: np.ndarray, coef, h: float, prm):
    """L(phi) without the source, and dL/dphi, at the interior (reading D3:
    no regularisation terms).
      Poisson     : L = Lap phi
      Hamiltonian : L = chi Lap Psi + A (chi^6 - 1) - 1/4 AA chi^-6, chi = 1 - kappa Psi
      CMC         : L = Lap xi - m2 xi"""
    lp, dlp = lap(phi, h)
    c = interior(phi)
    if kind == POISSON:
        return lp, dlp
    if kind == CMC:
        return lp - coef * c, dlp - coef
    kap = _kappa(prm)
    A = 1.5 * prm.a * prm.omega_m
    chi = 1.0 - kap * c
    chi2 = chi * chi
    chi5 = chi2 * chi2 * chi
    chi6 = chi5 * chi
    chim6 = 1.0 / chi6
    chim7 = chim6 / chi
    L = chi * lp + A * (chi6 - 1.0) - 0.25 * coef * chim6
    J = -kap * lp + chi * dlp - 6.0 * A * kap * chi5 - 1.5 * kap * coef * chim7
    return L, J


def _colour(n: int) -> np.ndarray:
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return (i + j + k) & 1


def rb_sweep(kind, phi, f, coef, h, prm) -> None:
    """One red-black sweep of the interior, even colour first.  A point's
    update reads only the other colour, so evaluating the operator on the whole
    interior and updating one colour is exactly the point-by-point sweep."""
    col = _colour(phi.shape[0] - 2)
    ph = interior(phi)
    for colour in (0, 1):
        L, J = op(kind, phi, coef, h, prm)
        m = col == colour
        ph[m] = ph[m] - (L[m] - f[m]) / J[m]


def residual(kind, phi, f, coef, h, prm) -> np.ndarray:
    return op(kind, phi, coef, h, prm)[0] - f


def restrict(x: np.ndarray) -> np.ndarray:
    """Mean of the 8 children (interior arrays), children summed in the order
    c = 0..7 with (dx, dy, dz) = (c & 1, (c >> 1) & 1, c >> 2)."""
    s = np.zeros(tuple(d // 2 for d in x.shape))
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, c >> 2
        s = s + x[dz::2, dy::2, dx::2]
    return s / 8.0


def prolong_add(e: np.ndarray, phi: np.ndarray) -> None:
    """Adds the cell-centred trilinear prolongation of the interior coarse
    correction e (m^3) to the interior of the padded fine array (2m+2)^3; the
    correction is continued oddly across every face (reading D4), per axis,
    so edge and corner values are products of reflections."""
    m = e.shape[0]
    ep = np.zeros((m + 2, m + 2, m + 2))
    interior(ep)[...] = e
    ep[0, :, :] = -ep[1, :, :]
    ep[-1, :, :] = -ep[-2, :, :]
    ep[:, 0, :] = -ep[:, 1, :]
    ep[:, -1, :] = -ep[:, -2, :]
    ep[:, :, 0] = -ep[:, :, 1]
    ep[:, :, -1] = -ep[:, :, -2]
    i = np.arange(2 * m)
    near = i // 2 + 1
    far = near + np.where(i & 1, 1, -1)
    v = np.zeros((2 * m, 2 * m, 2 * m))
    for c in range(8):
        ox, oy, oz = c & 1, (c >> 1) & 1, c >> 2
        w = (0.25 if ox else 0.75) * (0.25 if oy else 0.75) * (0.25 if oz else 0.75)
        v = v + w * ep[np.ix_(far if oz else near, far if oy else near, far if ox else near)]
    interior(phi)[...] += v


# ------------------------------------------------------------------ solver

class _Level:
    def __init__(self, phi, f, coef, h):
        self.phi, self.f, self.coef, self.h = phi, f, coef, h
        self.phi0 = None


def _vcycle(H: list, l: int, kind, prm, nu1, nu2) -> None:
    L = H[l]
    if l == len(H) - 1:
        for _ in range(COARSE_SWEEPS):
            rb_sweep(kind, L.phi, L.f, L.coef, L.h, prm)
        return
    for _ in range(nu1):
        rb_sweep(kind, L.phi, L.f, L.coef, L.h, prm)
    r = residual(kind, L.phi, L.f, L.coef, L.h, prm)
    C = H[l + 1]
    interior(C.phi)[...] = restrict(interior(L.phi))
    C.phi0 = interior(C.phi).copy()
    C.f = op(kind, C.phi, C.coef, C.h, prm)[0] - restrict(r)
    _vcycle(H, l + 1, kind, prm, nu1, nu2)
    prolong_add(interior(C.phi) - C.phi0, L.phi)
    for _ in range(nu2):
        rb_sweep(kind, L.phi, L.f, L.coef, L.h, prm)


def solve(kind, phi, f, coef, coarse_bnd, h, prm, nu1=2, nu2=2, max_cycles=100, rtol=1e-10):
    """FAS V-cycles on one patch.
      phi        : padded level-0 array: interior = guess, face cells = boundary values
      f, coef    : interior arrays (coef: AA for the Hamiltonian, m^2 for
                   CMC, None for Poisson)
      coarse_bnd : padded arrays of levels 1.. whose face cells hold those
                   levels' boundary values (their interiors are not used)
    Returns (phi, status, cycles, rel) with rel = rms(eps)/rms(f) at the start
    of the last cycle (the stopping test of the periodic solver)."""
    phi = np.array(phi, dtype=np.float64)
    n = phi.shape[0] - 2
    sizes = levels(n)
    assert len(coarse_bnd) == len(sizes) - 1
    if coef is None:
        coef = np.zeros((n, n, n))
    H = [_Level(phi, np.asarray(f, dtype=np.float64), np.asarray(coef, dtype=np.float64), h)]
    for l in range(1, len(sizes)):
        g = np.array(coarse_bnd[l - 1], dtype=np.float64)
        assert g.shape[0] == sizes[l] + 2
        H.append(_Level(g, None, restrict(H[l - 1].coef), h * (1 << l)))
    cyc, rel, st = 0, 0.0, OK
    fn = float(np.sqrt(np.mean(H[0].f * H[0].f)))
    while True:
        r = residual(kind, phi, H[0].f, H[0].coef, h, prm)
        rn = float(np.sqrt(np.mean(r * r)))
        rel = rn / (fn if fn > 0.0 else 1.0)
        if not np.isfinite(rel):
            st = ENAN
            break
        if rtol > 0.0 and (rel <= rtol or rn == 0.0):
            break
        if cyc >= max_cycles:
            st = ENOTCONV if rtol > 0.0 else OK
            break
        _vcycle(H, 0, kind, prm, nu1, nu2)
        cyc += 1
    return phi, st, cyc, rel


# ---------------------------------------------------------------- builders

def dcen(g: np.ndarray, axis: int, h: float) -> np.ndarray:
    """Central difference along x (0), y (1) or z (2) at the interior of a
    padded array."""
    if axis == 0:
        return (g[1:-1, 1:-1, 2:] - g[1:-1, 1:-1, :-2]) / (2.0 * h)
    if axis == 1:
        return (g[1:-1, 2:, 1:-1] - g[1:-1, :-2, 1:-1]) / (2.0 * h)
    return (g[2:, 1:-1, 1:-1] - g[:-2, 1:-1, 1:-1]) / (2.0 * h)


def div_quarter(gx, gy, gz, h) -> np.ndarray:
    """-1/4 d_j g^j (sources of U and b)."""
    return -0.25 * (dcen(gx, 0, h) + dcen(gy, 1, h) + dcen(gz, 2, h))


def _d2(U, a, b, h):
    """d_a d_b U at the interior: 3-point second difference on the diagonal,
    the 4-point diagonal-neighbour formula off it (sec. 4.3.1)."""
    n = U.shape[0] - 2

    def sh(dx, dy, dz):
        return U[1 + dz:1 + dz + n, 1 + dy:1 + dy + n, 1 + dx:1 + dx + n]

    e = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
    if a == b:
        d = e[a]
        return (sh(*d) - 2.0 * sh(0, 0, 0) + sh(-d[0], -d[1], -d[2])) / (h * h)
    p = tuple(e[a][k] + e[b][k] for k in range(3))
    q = tuple(e[a][k] - e[b][k] for k in range(3))
    return (sh(*p) + sh(-p[0], -p[1], -p[2]) - sh(*q) - sh(-q[0], -q[1], -q[2])) / (4.0 * h * h)


def build_Aij(V, U, h):
    """A_ij = d_iV_j + d_jV_i - 1/2 delta_ij d_kV^k + 2 d_i d_j U at the interior,
    packed (xx, yy, zz, xy, xz, yz), and AA = A_ij A^ij (sec. 4.3.1)."""
    n = U.shape[0] - 2
    pa, pb = (0, 1, 2, 0, 0, 1), (0, 1, 2, 1, 2, 2)
    divV = dcen(V[0], 0, h) + dcen(V[1], 1, h) + dcen(V[2], 2, h)
    A6 = np.empty((6, n, n, n))
    AA = np.zeros((n, n, n))
    for c in range(6):
        x, y = pa[c], pb[c]
        A = dcen(V[y], x, h) + dcen(V[x], y, h) + 2.0 * _d2(U, x, y, h)
        if x == y:
            A = A - 0.5 * divV
        A6[c] = A
        AA = AA + (1.0 if x == y else 2.0) * A * A
    return A6, AA


def build_cmc(psi, s0, sm, AA, prm):
    """m^2 = chi^-1 Q/(a^2 c^2) and the (unregularised) CMC source (sec. 4.3.2.2)."""
    a, c, om = prm.a, prm.c_tilde, prm.omega_m
    chi = 1.0 - _kappa(prm) * psi
    chi2 = chi * chi
    chi6 = chi2 * chi2 * chi2
    chim7 = 1.0 / (chi6 * chi)
    Q = 0.75 * a * om / chi * (s0 + 5.0 * chi6 + 2.0 * sm) + 0.875 * AA * chim7
    return Q / (chi * a * a * c * c), 1.5 * a * om / chi * (s0 - chi6 + sm) + AA * chim7


def build_shift_source(psi, xi, A6p, h, prm):
    """2 d_j[alpha chi^-6 A^ij] at the interior from padded Psi, xi and padded
    A_ij (6 components; the shells hold the ghost values)."""
    a, c = prm.a, prm.c_tilde
    chi = 1.0 - _kappa(prm) * psi
    chi2 = chi * chi
    chi6 = chi2 * chi2 * chi2
    alpha = 1.0 + (xi / chi) / (a * a * c * c)
    Ap = alpha / chi6 * A6p
    comp = ((0, 3, 4), (3, 1, 5), (4, 5, 2))
    out = []
    for row in range(3):
        s = dcen(Ap[comp[row][0]], 0, h) + dcen(Ap[comp[row][1]], 1, h) + dcen(Ap[comp[row][2]], 2, h)
        out.append(2.0 * s)
    return out


# ------------------------------------------------------------ whole patch

def solve_patch(parent: dict, parent_A6: np.ndarray, H: float, src: dict, n: int, h: float, origin,
                prm, nu1=2, nu2=2, max_cycles=100, rtol=1e-10, periodic: bool = True, return_A6: bool = False):
    """The ten equations on one patch in the order of the solution scheme
    (sec. 2.4), zero interior guesses, boundary values from the solved parent.
      parent    : the parent's ten solved fields by name (N^3: a periodic box,
                  or with periodic=False the interior of a parent patch, D6)
      parent_A6 : the parent's A_ij (6, N, N, N)
      src       : the patch's s0, sx, sy, sz, sm (interior, n^3)
      max_cycles: an int, or one count per field (exactly that many cycles
                  with rtol = 0)
    Returns (fields: name -> padded array with the face values, status,
    cycles[10], rel[10], AA) and, with return_A6, the patch's A_ij."""
    a, om = prm.a, prm.omega_m
    out, cycles, rels, status = {}, [0] * 10, [0.0] * 10, OK

    def run(name, kind, f, coef=None):
        nonlocal status
        g = boundary_of(parent[name], H, n, h, origin, periodic)
        phi = g[0].copy()
        k = FIELDS.index(name)
        mc = max_cycles[k] if hasattr(max_cycles, "__len__") else max_cycles
        phi, st, cyc, rel = solve(kind, phi, f, coef, g[1:], h, prm, nu1, nu2, mc, rtol)
        out[name], cycles[k], rels[k] = phi, cyc, rel
        if st != OK and status == OK:
            status = st

    def stencil_view(name):
        """The solved field with the parent at the outside cell centres (D5)."""
        v = sample_parent(parent[name], H, n, h, origin, periodic)
        interior(v)[...] = interior(out[name])
        return v

    for d, name in enumerate(("Vx", "Vy", "Vz")):
        run(name, POISSON, 3.0 * om * a * np.asarray(src[("sx", "sy", "sz")[d]], dtype=np.float64))
    V = [stencil_view(k) for k in ("Vx", "Vy", "Vz")]
    run("U", POISSON, div_quarter(V[0], V[1], V[2], h))
    A6, AA = build_Aij(V, stencil_view("U"), h)
    run("Psi", HAMILTONIAN, 1.5 * a * om * (np.asarray(src["s0"], dtype=np.float64) - 1.0), AA)
    m2, fxi = build_cmc(interior(out["Psi"]), src["s0"], src["sm"], AA, prm)
    run("xi", CMC, fxi, m2)
    A6p = np.stack([sample_parent(parent_A6[c], H, n, h, origin, periodic) for c in range(6)])
    A6p[:, 1:-1, 1:-1, 1:-1] = A6
    fB = build_shift_source(stencil_view("Psi"), stencil_view("xi"), A6p, h, prm)
    for d, name in enumerate(("Bx", "By", "Bz")):
        run(name, POISSON, fB[d])
    Bv = [stencil_view(k) for k in ("Bx", "By", "Bz")]
    run("b", POISSON, div_quarter(Bv[0], Bv[1], Bv[2], h))
    if return_A6:
        return out, status, cycles, rels, AA, A6
    return out, status, cycles, rels, AA
