/*
 * Plain FP64 CPU oracle for the elliptic constraint/gauge solve of the
 * constrained-ADM N-body method (Barrera-Hinojosa & Li 2019, "GRAMSES I").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * library: every formula below is restated here from the paper.
 *
 * It is deliberately plain: serial loops, one array per quantity, no blocking,
 * no fusion, no reordering beyond what the algorithm states.  Built with
 * `-O2 -ffp-contract=off` so that every product is rounded separately.
 *
 * What it computes (paper section 4, "Numerical implementation"):
 *   - CIC deposit of s0, s_l and the stress trace s_m (sec. 4.1.2, CIC
 *     equations; Lorentz factor W of sec. 4.4).
 *   - The ten field equations in the order of sec. 2.4's solution scheme:
 *       V_i  : Lap V_i = 3 Om a (s_i - <s_i>)              (sec. 4.3.1)
 *       U    : Lap U   = -1/4 d_j V^j
 *       A_ij = d_iV_j + d_jV_i - 1/2 delta_ij d_kV^k + 2 d_i d_j U
 *       Psi  : regularised Hamiltonian constraint         (sec. 4.3.2.1)
 *       xi   : regularised CMC lapse equation, xi = Phi chi (sec. 4.3.2.2)
 *       B^i  : Lap B^i = 2 d_j[alpha chi^-6 A^ij]
 *       b    : Lap b   = -1/4 d_j B^j
 *     with the 7-point Laplacian and 3-point central differences of
 *     sec. 4.3.1 and the 4-point cross derivative of U.
 *   - Each equation by FAS multigrid V-cycles (sec. 4.3.1: residual
 *     eps = L(phi) - f, coarse equation with restricted residual, correction
 *     by prolongation, all levels down to the coarsest), smoothed by
 *     red-black Gauss-Seidel with one pointwise Newton step per visit.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   R1 constant mode: every periodic fine-level solution is pinned to zero
 *      mean: the guess is pinned, and re-pinned after every V-cycle.
 *   R2 <F> (Hamiltonian) and <m^2 xi> (CMC) are evaluated once per cycle
 *      from the pinned iterate and held fixed for that cycle.
 *   R3 colour = (i+j+k) mod 2 on level-local indices, even colour first.
 *   R4 restriction = mean of the 8 children; prolongation = cell-centred
 *      trilinear (3/4 near, 1/4 far per axis); operator coefficients (A_ijA^ij
 *      for Psi, m^2 for xi) are restricted with the same operator.
 *   R5 coarsest level: halve while n/2 is even; there do 32 red-black sweeps,
 *      then remove the mean of the correction.
 *   R6 stop when rms(eps)/rms(f) <= rtol, evaluated at the start of a cycle;
 *      rtol <= 0 means "run exactly max_cycles cycles".
 *   R7 s_m is the stress trace gamma^ij s_ij with the particle's own
 *      chi (CIC-interpolated Psi): m a^-2 chi^-4 u.u/(W c) per particle.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double a;       /* fiducial scale factor */
    double omega_m; /* matter density parameter */
    double c_tilde; /* speed of light in code units, c/(L H0) */
} orc_params;

enum { ORC_POISSON = 0, ORC_HAMILTONIAN = 1, ORC_CMC = 2 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOTCONV = -3, ORC_ENAN = -4, ORC_ENOMEM = -5 };

/* ------------------------------------------------------------------ grid */

static long at(int n, int i, int j, int k)
{
    /* periodic wrap (offsets never exceed one box length), C order
     * [k][j][i] with i (x) fastest */
    if (i < 0) i += n; else if (i >= n) i -= n;
    if (j < 0) j += n; else if (j >= n) j -= n;
    if (k < 0) k += n; else if (k >= n) k -= n;
    return ((long)k * n + j) * n + i;
}

static double mean_of(const double *x, long N)
{
    double s = 0.0;
    for (long p = 0; p < N; ++p) s += x[p];
    return s / (double)N;
}

static double rms_of(const double *x, long N)
{
    double s = 0.0;
    for (long p = 0; p < N; ++p) s += x[p] * x[p];
    return sqrt(s / (double)N);
}

/* 7-point Laplacian, sec. 4.3.1 */
static double lap7(const double *phi, int n, double h, int i, int j, int k)
{
    double nb = phi[at(n, i + 1, j, k)] + phi[at(n, i - 1, j, k)]
              + phi[at(n, i, j + 1, k)] + phi[at(n, i, j - 1, k)]
              + phi[at(n, i, j, k + 1)] + phi[at(n, i, j, k - 1)];
    return (nb - 6.0 * phi[at(n, i, j, k)]) / (h * h);
}

/* central difference d_dir, sec. 4.3.1 (3-point stencil) */
static double dcen(const double *g, int n, double h, int dir, int i, int j, int k)
{
    int di = dir == 0, dj = dir == 1, dk = dir == 2;
    return (g[at(n, i + di, j + dj, k + dk)] - g[at(n, i - di, j - dj, k - dk)]) / (2.0 * h);
}

/* d_a d_b U: diagonal 3-point second difference, off-diagonal 4-point
 * diagonal-neighbour formula of sec. 4.3.1 */
static double d2(const double *U, int n, double h, int a, int b, int i, int j, int k)
{
    int e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (a == b) {
        return (U[at(n, i + e[a][0], j + e[a][1], k + e[a][2])] - 2.0 * U[at(n, i, j, k)]
                + U[at(n, i - e[a][0], j - e[a][1], k - e[a][2])]) / (h * h);
    }
    int pi = e[a][0] + e[b][0], pj = e[a][1] + e[b][1], pk = e[a][2] + e[b][2];
    int qi = e[a][0] - e[b][0], qj = e[a][1] - e[b][1], qk = e[a][2] - e[b][2];
    double upp = U[at(n, i + pi, j + pj, k + pk)];
    double umm = U[at(n, i - pi, j - pj, k - pk)];
    double upm = U[at(n, i + qi, j + qj, k + qk)];
    double ump = U[at(n, i - qi, j - qj, k - qk)];
    return (upp + umm - upm - ump) / (4.0 * h * h);
}

/* ------------------------------------------------------------- operators */

typedef struct {
    int kind;
    double kappa;  /* 1/(2 a^2 c^2): chi = 1 - kappa Psi */
    double A;      /* 3/2 a Om */
    double Fbar;   /* frozen <F>, Hamiltonian finest level only (else 0) */
    double fshift; /* frozen <f> + <m^2 xi>, CMC finest level only (else 0) */
} op_t;

/* L(phi) at one point (without the source) and its derivative with respect to
 * phi at that point, neighbours held fixed.
 *   Poisson     : L = Lap phi
 *   Hamiltonian : L = chi Lap Psi + A (chi^6 - 1) - 1/4 AA chi^-6 + Fbar chi
 *                 (sec. 4.3.2.1; Fbar term = regularisation, finest only)
 *   CMC         : L = Lap xi - m2 xi  (sec. 4.3.2.2) */
static double op_point(const op_t *op, const double *phi, const double *coef,
                       int n, double h, int i, int j, int k, double *dLdphi)
{
    long p = at(n, i, j, k);
    double lap = lap7(phi, n, h, i, j, k);
    if (op->kind == ORC_POISSON) {
        *dLdphi = -6.0 / (h * h);
        return lap;
    }
    if (op->kind == ORC_CMC) {
        double m2 = coef[p];
        *dLdphi = -6.0 / (h * h) - m2;
        return lap - m2 * phi[p];
    }
    /* Hamiltonian */
    double kap = op->kappa, A = op->A, AA = coef[p];
    double chi = 1.0 - kap * phi[p];
    double chi2 = chi * chi;
    double chi5 = chi2 * chi2 * chi;
    double chi6 = chi5 * chi;
    double chim6 = 1.0 / chi6;
    double chim7 = chim6 / chi;
    double L = chi * lap + A * (chi6 - 1.0) - 0.25 * AA * chim6 + op->Fbar * chi;
    /* d chi / d Psi = -kappa */
    *dLdphi = -kap * lap + chi * (-6.0 / (h * h)) - 6.0 * A * kap * chi5
              - 1.5 * kap * AA * chim7 - kap * op->Fbar;
    return L;
}

/* F of sec. 4.3.2.1 written with f = A (s0 - 1):
 * F = chi^-1 [A s0 - A chi^6] + 1/4 AA chi^-7 = (f - A (chi^6 - 1))/chi + AA chi^-7 / 4 */
static double ham_F(double kap, double A, double psi, double f, double AA)
{
    double chi = 1.0 - kap * psi;
    double chi2 = chi * chi;
    double chi6 = chi2 * chi2 * chi2;
    double chim7 = 1.0 / (chi6 * chi);
    return (f - A * (chi6 - 1.0)) / chi + 0.25 * AA * chim7;
}

/* one red-black sweep: even colour first, then odd (reading R3) */
static void rb_sweep(const op_t *op, double *phi, const double *f, const double *coef, int n, double h)
{
    for (int colour = 0; colour < 2; ++colour)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    if (((i + j + k) & 1) != colour) continue;
                    long p = at(n, i, j, k);
                    double J;
                    double L = op_point(op, phi, coef, n, h, i, j, k, &J);
                    double res = L - (f[p] - op->fshift);
                    phi[p] = phi[p] - res / J;
                }
}

static void residual(const op_t *op, const double *phi, const double *f, const double *coef,
                     int n, double h, double *r)
{
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long p = at(n, i, j, k);
                double J;
                r[p] = op_point(op, phi, coef, n, h, i, j, k, &J) - (f[p] - op->fshift);
            }
}

/* R: mean of the 8 children (reading R4) */
static void restrict8(const double *fine, int n, double *coarse)
{
    int m = n / 2;
    for (int K = 0; K < m; ++K)
        for (int J = 0; J < m; ++J)
            for (int I = 0; I < m; ++I) {
                double s = 0.0;
                for (int c = 0; c < 8; ++c)
                    s += fine[at(n, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2))];
                coarse[at(m, I, J, K)] = s / 8.0;
            }
}

/* P: cell-centred trilinear.  Fine cell 2I lies a quarter coarse cell below
 * the centre of coarse cell I, so it takes 3/4 of I and 1/4 of I-1; fine
 * cell 2I+1 takes 3/4 of I and 1/4 of I+1 (reading R4). Adds P(e) to fine. */
static void prolong_add(const double *e, int m, double *fine)
{
    int n = 2 * m;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int I = i / 2, J = j / 2, K = k / 2;
                int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                double v = 0.0;
                for (int c = 0; c < 8; ++c) {
                    int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                    double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
                    v += w * e[at(m, I + ox * si, J + oy * sj, K + oz * sk)];
                }
                fine[at(n, i, j, k)] += v;
            }
}

/* Cubic interpolation of a coarse m^3 field to the (2m)^3 cell-centred grid,
 * used only to spread a coarse-level initial guess (it is not the multigrid
 * prolongation).  Per dimension, a fine centre lies a quarter coarse cell
 * from the nearest coarse centre; the value there is the Lagrange cubic
 * through the four nearest coarse centres (periodic), and the 3-D value the
 * tensor product of the three 1-D rules, summed directly over 64 points. */
static void cubic_weights(int fine_index, int *first, double w[4])
{
    /* nodes at coarse centres first .. first+3, evaluation point t in node units */
    int I = fine_index / 2;
    double t;
    if (fine_index & 1) {
        *first = I - 1;
        t = 1.25; /* I + 1/4 */
    } else {
        *first = I - 2;
        t = 1.75; /* I - 1/4 */
    }
    for (int j = 0; j < 4; ++j) {
        double v = 1.0;
        for (int k = 0; k < 4; ++k)
            if (k != j) v *= (t - k) / (double)(j - k);
        w[j] = v;
    }
}

void orc_interp_cubic(int m, const double *coarse, double *fine)
{
    int n = 2 * m;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int fi, fj, fk;
                double wi[4], wj[4], wk[4];
                cubic_weights(i, &fi, wi);
                cubic_weights(j, &fj, wj);
                cubic_weights(k, &fk, wk);
                double v = 0.0;
                for (int c = 0; c < 4; ++c)
                    for (int b = 0; b < 4; ++b)
                        for (int a = 0; a < 4; ++a)
                            v += wi[a] * wj[b] * wk[c] * coarse[at(m, fi + a, fj + b, fk + c)];
                fine[at(n, i, j, k)] = v;
            }
}

/* --------------------------------------------------------------- multigrid */

#define ORC_MAXLEV 24
#define ORC_COARSE_SWEEPS 32

typedef struct {
    int nlev;
    int n[ORC_MAXLEV];
    double h[ORC_MAXLEV];
    double *phi[ORC_MAXLEV];  /* level 0: the caller's field */
    double *phi0[ORC_MAXLEV]; /* restricted iterate R phi (coarse levels) */
    double *f[ORC_MAXLEV];
    double *coef[ORC_MAXLEV];
    double *r[ORC_MAXLEV];
} hier_t;

/* number of levels: halve while n/2 is even (reading R5) */
int orc_num_levels(int n)
{
    int L = 1;
    while (n % 4 == 0) { n /= 2; ++L; }
    return L;
}

static int hier_alloc(hier_t *H, int n, double h)
{
    memset(H, 0, sizeof(*H));
    H->nlev = orc_num_levels(n);
    for (int l = 0; l < H->nlev; ++l) {
        H->n[l] = n >> l;
        H->h[l] = h * (double)(1 << l);
        long N = (long)H->n[l] * H->n[l] * H->n[l];
        H->phi0[l] = calloc(N, sizeof(double));
        H->f[l] = calloc(N, sizeof(double));
        H->coef[l] = calloc(N, sizeof(double));
        H->r[l] = calloc(N, sizeof(double));
        if (l > 0) H->phi[l] = calloc(N, sizeof(double));
        if (!H->phi0[l] || !H->f[l] || !H->coef[l] || !H->r[l] || (l > 0 && !H->phi[l])) return ORC_ENOMEM;
    }
    return ORC_OK;
}

static void hier_free(hier_t *H)
{
    for (int l = 0; l < H->nlev; ++l) {
        free(H->phi0[l]); free(H->f[l]); free(H->coef[l]); free(H->r[l]);
        if (l > 0) free(H->phi[l]);
    }
}

static void vcycle(hier_t *H, int l, const op_t *op_fine, const op_t *op_coarse, int nu1, int nu2)
{
    const op_t *op = (l == 0) ? op_fine : op_coarse;
    int n = H->n[l];
    double h = H->h[l];
    long N = (long)n * n * n;
    if (l == H->nlev - 1) {
        /* coarsest: 32 sweeps, then remove the mean of the correction */
        double *save = malloc(N * sizeof(double));
        memcpy(save, H->phi[l], N * sizeof(double));
        for (int s = 0; s < ORC_COARSE_SWEEPS; ++s) rb_sweep(op, H->phi[l], H->f[l], H->coef[l], n, h);
        double dm = 0.0;
        for (long p = 0; p < N; ++p) dm += H->phi[l][p] - save[p];
        dm /= (double)N;
        for (long p = 0; p < N; ++p) H->phi[l][p] -= dm;
        free(save);
        return;
    }
    for (int s = 0; s < nu1; ++s) rb_sweep(op, H->phi[l], H->f[l], H->coef[l], n, h);
    residual(op, H->phi[l], H->f[l], H->coef[l], n, h, H->r[l]);
    int m = H->n[l + 1];
    long M = (long)m * m * m;
    restrict8(H->phi[l], n, H->phi[l + 1]);
    memcpy(H->phi0[l + 1], H->phi[l + 1], M * sizeof(double));
    /* coarse source of the FAS equation: f^H = L^H(R phi) - R eps */
    double *Rr = malloc(M * sizeof(double));
    restrict8(H->r[l], n, Rr);
    for (int K = 0; K < m; ++K)
        for (int J = 0; J < m; ++J)
            for (int I = 0; I < m; ++I) {
                double d;
                long q = at(m, I, J, K);
                H->f[l + 1][q] = op_point(op_coarse, H->phi[l + 1], H->coef[l + 1], m, H->h[l + 1], I, J, K, &d) - Rr[q];
            }
    free(Rr);
    vcycle(H, l + 1, op_fine, op_coarse, nu1, nu2);
    double *e = malloc(M * sizeof(double));
    for (long q = 0; q < M; ++q) e[q] = H->phi[l + 1][q] - H->phi0[l + 1][q];
    prolong_add(e, m, H->phi[l]);
    free(e);
    for (int s = 0; s < nu2; ++s) rb_sweep(op, H->phi[l], H->f[l], H->coef[l], n, h);
}

typedef struct {
    int nu1, nu2, max_cycles;
    double rtol;
} orc_opts;

/* Solve one equation on a periodic n^3 box of spacing h.
 *   kind  : ORC_POISSON | ORC_HAMILTONIAN | ORC_CMC
 *   phi   : in = guess, out = solution (pinned to zero mean)
 *   f     : fine source (Hamiltonian: 3/2 a Om (s0-1); CMC: unregularised f)
 *   coef  : AA for the Hamiltonian, m^2 for CMC, ignored (may be NULL) for Poisson
 * Returns ORC_OK, ORC_ENOTCONV (max_cycles reached with rtol > 0) or ORC_ENAN. */
int orc_solve_equation(int n, double h, const orc_params *prm, int kind, double *phi,
                       const double *f, const double *coef, const orc_opts *o,
                       int *cycles_out, double *rel_out)
{
    if (n < 2 || (n & 1) || kind < 0 || kind > 2) return ORC_EINVAL;
    hier_t H;
    int st = hier_alloc(&H, n, h);
    if (st) { hier_free(&H); return st; }
    long N = (long)n * n * n;
    H.phi[0] = phi;
    memcpy(H.f[0], f, N * sizeof(double));
    if (kind != ORC_POISSON) {
        memcpy(H.coef[0], coef, N * sizeof(double));
        for (int l = 1; l < H.nlev; ++l) restrict8(H.coef[l - 1], H.n[l - 1], H.coef[l]);
    }
    op_t opf = {kind, 0.0, 0.0, 0.0, 0.0};
    opf.kappa = 1.0 / (2.0 * prm->a * prm->a * prm->c_tilde * prm->c_tilde);
    opf.A = 1.5 * prm->a * prm->omega_m;
    op_t opc = opf; /* coarse levels: unregularised */
    double fbar = (kind == ORC_CMC) ? mean_of(H.f[0], N) : 0.0;

    /* pin the guess (reading R1) */
    double mu = mean_of(phi, N);
    for (long p = 0; p < N; ++p) phi[p] -= mu;

    int cyc = 0;
    double rel = 0.0;
    double *feff = malloc(N * sizeof(double));
    st = ORC_OK;
    for (;;) {
        /* cycle start: frozen means (reading R2), residual, stopping test */
        if (kind == ORC_HAMILTONIAN) {
            double s = 0.0;
            for (long p = 0; p < N; ++p) s += ham_F(opf.kappa, opf.A, phi[p], H.f[0][p], H.coef[0][p]);
            opf.Fbar = s / (double)N;
        } else if (kind == ORC_CMC) {
            double s = 0.0;
            for (long p = 0; p < N; ++p) s += H.coef[0][p] * phi[p];
            opf.fshift = fbar + s / (double)N;
        }
        residual(&opf, phi, H.f[0], H.coef[0], n, h, H.r[0]);
        for (long p = 0; p < N; ++p) feff[p] = H.f[0][p] - opf.fshift;
        double rn = rms_of(H.r[0], N), fn = rms_of(feff, N);
        rel = rn / (fn > 0.0 ? fn : 1.0);
        if (!isfinite(rel)) { st = ORC_ENAN; break; }
        if (o->rtol > 0.0 && (rel <= o->rtol || rn == 0.0)) break;
        if (cyc >= o->max_cycles) { st = (o->rtol > 0.0) ? ORC_ENOTCONV : ORC_OK; break; }
        vcycle(&H, 0, &opf, &opc, o->nu1, o->nu2);
        mu = mean_of(phi, N);
        for (long p = 0; p < N; ++p) phi[p] -= mu;
        ++cyc;
    }
    free(feff);
    hier_free(&H);
    if (cycles_out) *cycles_out = cyc;
    if (rel_out) *rel_out = rel;
    return st;
}

/* Exposed single steps, for step-by-step comparisons.  `Fbar` and `fshift`
 * are the frozen scalars of the operator (0 on coarse levels). */
void orc_rb_sweep(int n, double h, const orc_params *prm, int kind, double Fbar, double fshift,
                  double *phi, const double *f, const double *coef)
{
    op_t op = {kind, 1.0 / (2.0 * prm->a * prm->a * prm->c_tilde * prm->c_tilde),
               1.5 * prm->a * prm->omega_m, Fbar, fshift};
    rb_sweep(&op, phi, f, coef, n, h);
}

void orc_residual(int n, double h, const orc_params *prm, int kind, double Fbar, double fshift,
                  const double *phi, const double *f, const double *coef, double *r)
{
    op_t op = {kind, 1.0 / (2.0 * prm->a * prm->a * prm->c_tilde * prm->c_tilde),
               1.5 * prm->a * prm->omega_m, Fbar, fshift};
    residual(&op, phi, f, coef, n, h, r);
}

void orc_restrict(int n, const double *fine, double *coarse) { restrict8(fine, n, coarse); }

void orc_prolong_add(int m, const double *e, double *fine) { prolong_add(e, m, fine); }

/* ------------------------------------------------------------ CIC deposit */

/* Cloud-in-cell deposit (sec. 4.1.2), cell-centred weights with periodic wrap.
 * Per particle: chi_p = 1 - kappa * (CIC-interpolated Psi^n),
 * W^2 = c^2 + a^-2 chi_p^-4 sum_l u_l^2   (Lorentz factor, sec. 4.4),
 * s0 += w m W/(c h^3), s_l += w m u_l/(c h^3) and the stress trace
 * s_m = gamma^ij s_ij += w m a^-2 chi^-4 u.u/(W c h^3)  (s_ij ~ u_i u_j/(W c)).
 * pos, u: [np][3]; psi may be NULL (Psi^n = 0). Outputs are overwritten. */
void orc_cic_deposit(int n, const orc_params *prm, long np, const double *pos, const double *u,
                     double mass, const double *psi, double *s0, double *sx, double *sy, double *sz,
                     double *sm)
{
    long N = (long)n * n * n;
    double h = 1.0 / n, c = prm->c_tilde, a = prm->a;
    double kap = 1.0 / (2.0 * a * a * c * c);
    double vol = h * h * h;
    memset(s0, 0, N * sizeof(double));
    memset(sx, 0, N * sizeof(double));
    memset(sy, 0, N * sizeof(double));
    memset(sz, 0, N * sizeof(double));
    memset(sm, 0, N * sizeof(double));
    for (long q = 0; q < np; ++q) {
        int i0[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
            double g = pos[3 * q + d] / h - 0.5;
            double fl = floor(g);
            i0[d] = (int)fl;
            t[d] = g - fl;
        }
        double psi_p = 0.0;
        if (psi) {
            for (int cc = 0; cc < 8; ++cc) {
                int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
                double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
                psi_p += w * psi[at(n, i0[0] + ox, i0[1] + oy, i0[2] + oz)];
            }
        }
        double chi = 1.0 - kap * psi_p;
        double chi2 = chi * chi;
        double u2 = u[3 * q] * u[3 * q] + u[3 * q + 1] * u[3 * q + 1] + u[3 * q + 2] * u[3 * q + 2];
        double g_uu = u2 / (a * a * chi2 * chi2); /* gamma^ij u_i u_j */
        double W = sqrt(c * c + g_uu);
        double q0 = mass * W / (c * vol);
        double qx = mass * u[3 * q] / (c * vol);
        double qy = mass * u[3 * q + 1] / (c * vol);
        double qz = mass * u[3 * q + 2] / (c * vol);
        double qm = mass * g_uu / (W * c * vol); /* gamma^ij s_ij, s_ij ~ u_i u_j/(W c) */
        for (int cc = 0; cc < 8; ++cc) {
            int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
            double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
            long p = at(n, i0[0] + ox, i0[1] + oy, i0[2] + oz);
            s0[p] += w * q0;
            sx[p] += w * qx;
            sy[p] += w * qy;
            sz[p] += w * qz;
            sm[p] += w * qm;
        }
    }
}

/* --------------------------------------------------------- source builders */

/* A_ij (sec. 4.3.1) from V_i and U; outputs the six components
 * (xx, yy, zz, xy, xz, yz) and AA = A_ij A^ij (conformally flat, so
 * A^ij = A_ij). */
void orc_build_Aij(int n, const double *Vx, const double *Vy, const double *Vz, const double *U,
                   double *Aij6, double *AA)
{
    long N = (long)n * n * n;
    double h = 1.0 / n;
    const double *V[3] = {Vx, Vy, Vz};
    int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long p = at(n, i, j, k);
                double divV = dcen(V[0], n, h, 0, i, j, k) + dcen(V[1], n, h, 1, i, j, k)
                            + dcen(V[2], n, h, 2, i, j, k);
                double s = 0.0;
                for (int c = 0; c < 6; ++c) {
                    int x = pa[c], y = pb[c];
                    double A = dcen(V[y], n, h, x, i, j, k) + dcen(V[x], n, h, y, i, j, k)
                             + 2.0 * d2(U, n, h, x, y, i, j, k);
                    if (x == y) A -= 0.5 * divV;
                    Aij6[c * N + p] = A;
                    s += (x == y ? 1.0 : 2.0) * A * A;
                }
                AA[p] = s;
            }
}

/* -1/4 d_j g^j (sources of U and b) */
void orc_build_div_quarter(int n, const double *gx, const double *gy, const double *gz, double *f)
{
    double h = 1.0 / n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                f[at(n, i, j, k)] = -0.25 * (dcen(gx, n, h, 0, i, j, k) + dcen(gy, n, h, 1, i, j, k)
                                             + dcen(gz, n, h, 2, i, j, k));
}

/* CMC operator coefficient m^2 = chi^-1 Q/(a^2 c^2) and source f (sec. 4.3.2.2,
 * Q of the code-unit CMC equation) from the solved Psi. */
void orc_build_cmc(int n, const orc_params *prm, const double *psi, const double *s0,
                   const double *sm, const double *AA, double *m2, double *f)
{
    long N = (long)n * n * n;
    double a = prm->a, c = prm->c_tilde, om = prm->omega_m;
    double kap = 1.0 / (2.0 * a * a * c * c);
    for (long p = 0; p < N; ++p) {
        double chi = 1.0 - kap * psi[p];
        double chi2 = chi * chi, chi6 = chi2 * chi2 * chi2;
        double chim7 = 1.0 / (chi6 * chi);
        double Q = 0.75 * a * om / chi * (s0[p] + 5.0 * chi6 + 2.0 * sm[p]) + 0.875 * AA[p] * chim7;
        m2[p] = Q / (chi * a * a * c * c);
        f[p] = 1.5 * a * om / chi * (s0[p] - chi6 + sm[p]) + AA[p] * chim7;
    }
}

/* Source of B^i: 2 d_j[alpha chi^-6 A^ij], alpha = 1 + Phi/(a^2 c^2),
 * Phi = xi/chi (sec. 4.3.1, the primed A of the divergence formula). */
void orc_build_shift_source(int n, const orc_params *prm, const double *psi, const double *xi,
                            const double *Aij6, double *fBx, double *fBy, double *fBz)
{
    long N = (long)n * n * n;
    double h = 1.0 / n, a = prm->a, c = prm->c_tilde;
    double kap = 1.0 / (2.0 * a * a * c * c);
    double *Ap = malloc(6 * N * sizeof(double));
    for (long p = 0; p < N; ++p) {
        double chi = 1.0 - kap * psi[p];
        double chi2 = chi * chi, chi6 = chi2 * chi2 * chi2;
        double alpha = 1.0 + (xi[p] / chi) / (a * a * c * c);
        for (int cc = 0; cc < 6; ++cc) Ap[cc * N + p] = alpha / chi6 * Aij6[cc * N + p];
    }
    /* component index of (row, col) in the (xx,yy,zz,xy,xz,yz) packing */
    int comp[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    double *out[3] = {fBx, fBy, fBz};
    for (int row = 0; row < 3; ++row)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int col = 0; col < 3; ++col) s += dcen(Ap + comp[row][col] * N, n, h, col, i, j, k);
                    out[row][at(n, i, j, k)] = 2.0 * s;
                }
    free(Ap);
}

/* ---------------------------------------------------------- whole solve */

enum { F_VX, F_VY, F_VZ, F_U, F_PSI, F_XI, F_BX, F_BY, F_BZ, F_B, F_NFIELD };

/* Solve the ten equations in the order of the solution scheme (sec. 2.4):
 * V_i -> U -> (A_ij, AA) -> Psi -> xi -> B^i -> b.
 *   fields[10]: in = guesses, out = solutions (each n^3, unit box, h = 1/n)
 *   max_cycles[10], rtol: per-field cycle cap and tolerance (rtol <= 0: run
 *   exactly max_cycles[f] cycles).  AA (n^3) receives A_ij A^ij.
 * Returns the first non-OK status, after filling cycles[] and rel[]. */
int orc_solve_all(int n, const orc_params *prm, const double *s0, const double *sx,
                  const double *sy, const double *sz, const double *sm, double **fields,
                  int nu1, int nu2, const int *max_cycles, double rtol, int *cycles, double *rel,
                  double *AA)
{
    if (n < 2 || (n & 1)) return ORC_EINVAL;
    long N = (long)n * n * n;
    double h = 1.0 / n, a = prm->a, om = prm->omega_m;
    double *f = malloc(N * sizeof(double));
    double *coef = malloc(N * sizeof(double));
    double *Aij6 = malloc(6 * N * sizeof(double));
    double *fB[3] = {malloc(N * sizeof(double)), malloc(N * sizeof(double)), malloc(N * sizeof(double))};
    int first_bad = ORC_OK, st;
    orc_opts o = {nu1, nu2, 0, rtol};
    const double *s_i[3] = {sx, sy, sz};
#define SOLVE(fid, kind, src, cf)                                                            \
    do {                                                                                     \
        o.max_cycles = max_cycles[fid];                                                      \
        st = orc_solve_equation(n, h, prm, kind, fields[fid], src, cf, &o, &cycles[fid], &rel[fid]); \
        if (st && !first_bad) first_bad = st;                                                \
    } while (0)

    /* 1. V_i: Lap V_i = 3 Om a (s_i - <s_i>)  (mean removed: cyclic property) */
    for (int d = 0; d < 3; ++d) {
        double m = mean_of(s_i[d], N);
        for (long p = 0; p < N; ++p) f[p] = 3.0 * om * a * (s_i[d][p] - m);
        SOLVE(F_VX + d, ORC_POISSON, f, NULL);
    }
    /* 2. U: Lap U = -1/4 d_j V^j */
    orc_build_div_quarter(n, fields[F_VX], fields[F_VY], fields[F_VZ], f);
    SOLVE(F_U, ORC_POISSON, f, NULL);
    /* 3. A_ij and AA */
    orc_build_Aij(n, fields[F_VX], fields[F_VY], fields[F_VZ], fields[F_U], Aij6, AA);
    /* 4. Psi: Hamiltonian constraint, f = 3/2 a Om (s0 - 1), coefficient AA */
    for (long p = 0; p < N; ++p) f[p] = 1.5 * a * om * (s0[p] - 1.0);
    SOLVE(F_PSI, ORC_HAMILTONIAN, f, AA);
    /* 5. xi: CMC lapse equation with m^2 and f built from the solved Psi */
    orc_build_cmc(n, prm, fields[F_PSI], s0, sm, AA, coef, f);
    SOLVE(F_XI, ORC_CMC, f, coef);
    /* 6. B^i: Lap B^i = 2 d_j[alpha chi^-6 A^ij] */
    orc_build_shift_source(n, prm, fields[F_PSI], fields[F_XI], Aij6, fB[0], fB[1], fB[2]);
    for (int d = 0; d < 3; ++d) SOLVE(F_BX + d, ORC_POISSON, fB[d], NULL);
    /* 7. b: Lap b = -1/4 d_j B^j */
    orc_build_div_quarter(n, fields[F_BX], fields[F_BY], fields[F_BZ], f);
    SOLVE(F_B, ORC_POISSON, f, NULL);
#undef SOLVE
    free(f); free(coef); free(Aij6); free(fB[0]); free(fB[1]); free(fB[2]);
    return first_bad;
}

/* Derived fields after the solve: Phi = xi/chi and beta^i = B^i + d_i b. */
void orc_derived(int n, const orc_params *prm, const double *psi, const double *xi,
                 const double *Bx, const double *By, const double *Bz, const double *b,
                 double *Phi, double *betax, double *betay, double *betaz)
{
    long N = (long)n * n * n;
    double h = 1.0 / n;
    double kap = 1.0 / (2.0 * prm->a * prm->a * prm->c_tilde * prm->c_tilde);
    for (long p = 0; p < N; ++p) Phi[p] = xi[p] / (1.0 - kap * psi[p]);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                long p = at(n, i, j, k);
                betax[p] = Bx[p] + dcen(b, n, h, 0, i, j, k);
                betay[p] = By[p] + dcen(b, n, h, 1, i, j, k);
                betaz[p] = Bz[p] + dcen(b, n, h, 2, i, j, k);
            }
}

/* The stopping quantity of a given (pinned) iterate, as evaluated at the
 * start of a cycle: frozen means from phi, then rms(eps)/rms(f - fshift).
 * Used to check full-size results where a complete oracle solve is too slow. */
double orc_cycle_residual(int n, double h, const orc_params *prm, int kind, const double *phi,
                          const double *f, const double *coef)
{
    long N = (long)n * n * n;
    op_t op = {kind, 1.0 / (2.0 * prm->a * prm->a * prm->c_tilde * prm->c_tilde),
               1.5 * prm->a * prm->omega_m, 0.0, 0.0};
    if (kind == ORC_HAMILTONIAN) {
        double s = 0.0;
        for (long p = 0; p < N; ++p) s += ham_F(op.kappa, op.A, phi[p], f[p], coef[p]);
        op.Fbar = s / (double)N;
    } else if (kind == ORC_CMC) {
        double s = 0.0;
        for (long p = 0; p < N; ++p) s += coef[p] * phi[p];
        op.fshift = mean_of(f, N) + s / (double)N;
    }
    double *r = malloc(N * sizeof(double));
    double *fe = malloc(N * sizeof(double));
    residual(&op, phi, f, coef, n, h, r);
    for (long p = 0; p < N; ++p) fe[p] = f[p] - op.fshift;
    double rn = rms_of(r, N), fn = rms_of(fe, N);
    free(r);
    free(fe);
    return rn / (fn > 0.0 ? fn : 1.0);
}

/* ------------------------------------------------ particle evolution (N-body) */

/* Readings of sec. 4.4 (particles evolution) and of the leapfrog of the
 * appendix on time evolution:
 *   - the metric quantities at a particle are the cloud-in-cell interpolation
 *     (the deposit's cell-centred weights and periodic wrap) of the grid
 *     values: Phi, Psi, beta^i and their 3-point central-difference gradients
 *     d_i Phi, d_i Psi, d_i beta^j (sec. 4.3.1 difference stencil);
 *   - W^2 = c^2 + a^-2 chi^-4 u.u with chi = 1 - Psi/(2 a^2 c^2) from the
 *     interpolated Psi and the particle's current u;
 *   - the kick splits F_i = sum_j c_j (f_j)_i into five substeps, each taking
 *     c_j from the velocity as updated by the substeps before it, the f_j
 *     (gradients at the particle) fixed during the kick;
 *   - the drift uses the fields at the old position and the given u. */
enum { ORC_KICK_FORWARD = 0, ORC_KICK_REVERSE = 1 };

typedef struct {
    double Phi, Psi, beta[3];
    double dPhi[3], dPsi[3];
    double dbeta[3][3]; /* dbeta[i][j] = d_i beta^j */
} pfield_t;

static void particle_fields(int n, const double *Phi, const double *Psi, const double *const beta[3],
                            const double *x, pfield_t *F)
{
    double h = 1.0 / n;
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        double g = x[d] / h - 0.5;
        double fl = floor(g);
        i0[d] = (int)fl;
        t[d] = g - fl;
    }
    memset(F, 0, sizeof *F);
    for (int cc = 0; cc < 8; ++cc) {
        int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        /* corner indices, wrapped once so that the stencil offsets stay within one box length */
        int ci = i0[0] + ox, cj = i0[1] + oy, ck = i0[2] + oz;
        ci = (ci % n + n) % n;
        cj = (cj % n + n) % n;
        ck = (ck % n + n) % n;
        long p = at(n, ci, cj, ck);
        F->Phi += w * Phi[p];
        F->Psi += w * Psi[p];
        for (int d = 0; d < 3; ++d) {
            F->beta[d] += w * beta[d][p];
            F->dPhi[d] += w * dcen(Phi, n, h, d, ci, cj, ck);
            F->dPsi[d] += w * dcen(Psi, n, h, d, ci, cj, ck);
            for (int j = 0; j < 3; ++j) F->dbeta[d][j] += w * dcen(beta[j], n, h, d, ci, cj, ck);
        }
    }
}

static double lorentz_W(const orc_params *prm, double Psi, const double u[3])
{
    double a = prm->a, c = prm->c_tilde;
    double chi = 1.0 - Psi / (2.0 * a * a * c * c);
    double chi2 = chi * chi;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return sqrt(c * c + uu / (a * a * chi2 * chi2));
}

/* One kick of length dt for np particles (sec. 4.4): u_i += dt c_j (f_j)_i for
 * the five force contributions
 *   j = 1, 2, 3: c_j = -u_j,  (f_j)_i = -d_i beta^j
 *   j = 4:       c_4 = (W^2 - c^2)/(W c) (1 + Phi/(a^2c^2))/(1 - Psi/(2a^2c^2)),  (f_4)_i = -d_i Psi
 *   j = 5:       c_5 = W/c,  (f_5)_i = -d_i Phi
 * in the order 1..5 (ORC_KICK_FORWARD: the synchronising second kick, the
 * dominant term last) or 5..1 (ORC_KICK_REVERSE: the first kick).
 * Phi, Psi, beta: grid fields (n^3); pos, u: [np][3]. */
void orc_kick(int n, const orc_params *prm, const double *Phi, const double *Psi, const double *bx,
              const double *by, const double *bz, long np, const double *pos, double *u, double dt, int order)
{
    const double *beta[3] = {bx, by, bz};
    double a = prm->a, c = prm->c_tilde;
    for (long q = 0; q < np; ++q) {
        pfield_t F;
        particle_fields(n, Phi, Psi, beta, pos + 3 * q, &F);
        double *uq = u + 3 * q;
        for (int s = 0; s < 5; ++s) {
            int j = order == ORC_KICK_FORWARD ? s + 1 : 5 - s;
            double cj, f[3];
            if (j <= 3) {
                cj = -uq[j - 1];
                for (int i = 0; i < 3; ++i) f[i] = -F.dbeta[i][j - 1];
            } else {
                double W = lorentz_W(prm, F.Psi, uq);
                if (j == 4) {
                    cj = (W * W - c * c) / (W * c) * (1.0 + F.Phi / (a * a * c * c))
                         / (1.0 - F.Psi / (2.0 * a * a * c * c));
                    for (int i = 0; i < 3; ++i) f[i] = -F.dPsi[i];
                } else {
                    cj = W / c;
                    for (int i = 0; i < 3; ++i) f[i] = -F.dPhi[i];
                }
            }
            for (int i = 0; i < 3; ++i) uq[i] += dt * cj * f[i];
        }
    }
}

/* Drift (sec. 4.4): x^i += dt V^i,
 * V^i = (1 + Phi/(a^2c^2)) (1 - Psi/(2a^2c^2))^-4 (c/W) u_i - beta^i,
 * with the fields at the old position; positions wrapped into [0, 1). */
void orc_drift(int n, const orc_params *prm, const double *Phi, const double *Psi, const double *bx,
               const double *by, const double *bz, long np, double *pos, const double *u, double dt)
{
    const double *beta[3] = {bx, by, bz};
    double a = prm->a, c = prm->c_tilde;
    for (long q = 0; q < np; ++q) {
        pfield_t F;
        double *x = pos + 3 * q;
        const double *uq = u + 3 * q;
        particle_fields(n, Phi, Psi, beta, x, &F);
        double W = lorentz_W(prm, F.Psi, uq);
        double chi = 1.0 - F.Psi / (2.0 * a * a * c * c);
        double chi2 = chi * chi;
        double fac = (1.0 + F.Phi / (a * a * c * c)) / (chi2 * chi2) * (c / W);
        for (int d = 0; d < 3; ++d) {
            double v = fac * uq[d] - F.beta[d];
            double y = x[d] + dt * v;
            y -= floor(y);
            if (y >= 1.0) y = 0.0;
            x[d] = y;
        }
    }
}

/* Newtonian potential and kick (the temporary synchronisation option of
 * sec. 4.5 and of the appendix on time evolution): Phi_N solves the code-unit
 * Newtonian Poisson equation Lap Phi_N = 3/2 a Om (s0 - <s0>) (the weak-field,
 * chi -> 1 limit of the Hamiltonian constraint's source; the mean is removed
 * for periodic solvability, as sec. 4.3.1 does for the momentum source) by the
 * Poisson V-cycles to rtol, pinned to zero mean; then u_i -= dt d_i Phi_N at
 * every particle (the CIC interpolation of the central difference).  phiN
 * (n^3) receives the potential.  Returns the solve's status. */
int orc_newtonian_kick(int n, const orc_params *prm, const double *s0, double *phiN, long np, const double *pos,
                       double *u, double dt, double rtol, int max_cycles, int *cycles)
{
    long N = (long)n * n * n;
    double A = 1.5 * prm->a * prm->omega_m;
    double *f = malloc(N * sizeof(double));
    if (!f) return ORC_ENOMEM;
    /* A (s0 - 1), then minus its own mean: the same source as A (s0 - <s0>),
     * with the mean taken of the small deviations (no cancellation against 1) */
    for (long p = 0; p < N; ++p) f[p] = A * (s0[p] - 1.0);
    double fm = mean_of(f, N);
    for (long p = 0; p < N; ++p) f[p] -= fm;
    double rel = 0.0;
    memset(phiN, 0, N * sizeof(double));
    orc_opts o = {2, 2, max_cycles, rtol};
    int st = orc_solve_equation(n, 1.0 / n, prm, ORC_POISSON, phiN, f, NULL, &o, cycles, &rel);
    free(f);
    double *zero = calloc((size_t)N, sizeof(double));
    if (!zero) return ORC_ENOMEM;
    const double *beta[3] = {zero, zero, zero};
    for (long q = 0; q < np; ++q) {
        pfield_t F;
        particle_fields(n, phiN, zero, beta, pos + 3 * q, &F);
        for (int d = 0; d < 3; ++d) u[3 * q + d] -= dt * F.dPhi[d];
    }
    free(zero);
    return st;
}
