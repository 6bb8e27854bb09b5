// Per-point device arithmetic of the source and coefficient builders
// (paper sec. 4.3.1: 3-point central differences, the 4-point cross
// derivative of U, A_ij; sec. 4.3.2.2: Q, m2 and the CMC source; sec. 4.3.1:
// the shift source 2 d_j[alpha chi^-6 A^ij]), shared by the single-grid and
// batched kernels and the refinement patches, through field accessors.
#pragma once

#include "stencil_ops.h"

namespace grmg {
namespace detail {

// Field accessors: the value of a field at cell (i,j,k), which may lie one
// cell outside the box.  A periodic box wraps; a refinement patch reads its
// own cells inside and the parent's field outside (see patch_ops.h).
struct PeriodicField {
    const double *p;
    int n;
    __device__ __forceinline__ double operator()(int i, int j, int k) const
    {
        return p[lin(wrapi(i, n), wrapi(j, n), wrapi(k, n), n)];
    }
};

// Central difference of g along `dir` at (i,j,k): (g_+ - g_-)/(2h).
template <class F>
__device__ __forceinline__ double dcen_f(const F &g, int dir, int i, int j, int k, double inv2h)
{
    const int di = dir == 0, dj = dir == 1, dk = dir == 2;
    return (g(i + di, j + dj, k + dk) - g(i - di, j - dj, k - dk)) * inv2h;
}

// -1/4 d_j g^j
template <class F>
__device__ __forceinline__ double div_quarter_f(const F &gx, const F &gy, const F &gz, int i, int j, int k,
                                                double inv2h)
{
    return -0.25 * (dcen_f(gx, 0, i, j, k, inv2h) + dcen_f(gy, 1, i, j, k, inv2h) + dcen_f(gz, 2, i, j, k, inv2h));
}

// A_ij = d_iV_j + d_jV_i - 1/2 delta_ij d_kV^k + 2 d_i d_j U, packed (xx,yy,zz,xy,xz,yz);
// diagonal d_i d_i U: 3-point, off-diagonal: 4-point diagonal-neighbour formula.
// Returns A_ij A^ij (conformally flat: A^ij = A_ij).
template <class F>
__device__ __forceinline__ double aij_f(const F &Vx, const F &Vy, const F &Vz, const F &U, int i, int j, int k,
                                        double h, double (&A)[6])
{
    const double inv2h = 1.0 / (2.0 * h), invh2 = 1.0 / (h * h), inv4h2 = 1.0 / (4.0 * h * h);
    const F *V[3] = {&Vx, &Vy, &Vz};
    double dV[3][3]; // dV[a][b] = d_a V_b
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dV[a][b] = dcen_f(*V[b], a, i, j, k, inv2h);
    const double divV = dV[0][0] + dV[1][1] + dV[2][2];
    const double u0 = U(i, j, k);
    const double uxx = (U(i + 1, j, k) - 2.0 * u0 + U(i - 1, j, k)) * invh2;
    const double uyy = (U(i, j + 1, k) - 2.0 * u0 + U(i, j - 1, k)) * invh2;
    const double uzz = (U(i, j, k + 1) - 2.0 * u0 + U(i, j, k - 1)) * invh2;
    const double uxy = (U(i + 1, j + 1, k) + U(i - 1, j - 1, k) - U(i + 1, j - 1, k) - U(i - 1, j + 1, k)) * inv4h2;
    const double uxz = (U(i + 1, j, k + 1) + U(i - 1, j, k - 1) - U(i + 1, j, k - 1) - U(i - 1, j, k + 1)) * inv4h2;
    const double uyz = (U(i, j + 1, k + 1) + U(i, j - 1, k - 1) - U(i, j + 1, k - 1) - U(i, j - 1, k + 1)) * inv4h2;
    A[0] = 2.0 * dV[0][0] + 2.0 * uxx - 0.5 * divV;
    A[1] = 2.0 * dV[1][1] + 2.0 * uyy - 0.5 * divV;
    A[2] = 2.0 * dV[2][2] + 2.0 * uzz - 0.5 * divV;
    A[3] = dV[0][1] + dV[1][0] + 2.0 * uxy;
    A[4] = dV[0][2] + dV[2][0] + 2.0 * uxz;
    A[5] = dV[1][2] + dV[2][1] + 2.0 * uyz;
    return A[0] * A[0] + A[1] * A[1] + A[2] * A[2] + 2.0 * (A[3] * A[3] + A[4] * A[4] + A[5] * A[5]);
}

// periodic forms
__device__ __forceinline__ double dcen(const double *__restrict__ g, int dir, int i, int j, int k, int n,
                                       double inv2h)
{
    return dcen_f(PeriodicField{g, n}, dir, i, j, k, inv2h);
}

__device__ __forceinline__ double div_quarter_point(const double *__restrict__ gx, const double *__restrict__ gy,
                                                    const double *__restrict__ gz, int i, int j, int k, int n,
                                                    double inv2h)
{
    return div_quarter_f(PeriodicField{gx, n}, PeriodicField{gy, n}, PeriodicField{gz, n}, i, j, k, inv2h);
}

__device__ __forceinline__ double aij_point(const double *__restrict__ Vx, const double *__restrict__ Vy,
                                            const double *__restrict__ Vz, const double *__restrict__ U, int i,
                                            int j, int k, int n, double h, double (&A)[6])
{
    return aij_f(PeriodicField{Vx, n}, PeriodicField{Vy, n}, PeriodicField{Vz, n}, PeriodicField{U, n}, i, j, k, h,
                 A);
}

// CMC coefficient m2 = chi^-1 Q/(a^2c^2) and source
// f = 3/2 a Om chi^-1 [s0 - chi^6 + s_m] + AA chi^-7, with
// Q = 3/4 a Om chi^-1 [s0 + 5 chi^6 + 2 s_m] + 7/8 AA chi^-7.
__device__ __forceinline__ void cmc_point(double psi, double s0, double sm, double AA, double a, double om, double c,
                                          double &m2, double &f)
{
    const double kap = 1.0 / (2.0 * a * a * c * c);
    const double chi = 1.0 - kap * psi;
    const double chi2 = chi * chi, chi6 = chi2 * chi2 * chi2;
    const double chim7 = 1.0 / (chi6 * chi);
    const double Q = 0.75 * a * om / chi * (s0 + 5.0 * chi6 + 2.0 * sm) + 0.875 * AA * chim7;
    m2 = Q / (chi * a * a * c * c);
    f = 1.5 * a * om / chi * (s0 - chi6 + sm) + AA * chim7;
}

// f_B^i = 2 sum_j d_j[alpha chi^-6 A_ij], alpha = 1 + (xi/chi)/(a^2c^2).
template <class F>
__device__ __forceinline__ void shift_source_f(const F &psi, const F &xi, const F *A6, int i, int j, int k,
                                               double h, double a, double c, double (&out)[3])
{
    const double kap = 1.0 / (2.0 * a * a * c * c), ia2c2 = 1.0 / (a * a * c * c), inv2h = 1.0 / (2.0 * h);
    const int comp[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}}; // (row, col) -> packed component
    out[0] = out[1] = out[2] = 0.0;
    for (int col = 0; col < 3; ++col) {
        const int di = col == 0, dj = col == 1, dk = col == 2;
        double gfac[2];
        for (int s = 0; s < 2; ++s) {
            const int sg = s == 0 ? 1 : -1;
            const double ps = psi(i + sg * di, j + sg * dj, k + sg * dk);
            const double chi = 1.0 - kap * ps;
            const double chi2 = chi * chi, chi6 = chi2 * chi2 * chi2;
            const double alpha = 1.0 + (xi(i + sg * di, j + sg * dj, k + sg * dk) / chi) * ia2c2;
            gfac[s] = alpha / chi6;
        }
        for (int row = 0; row < 3; ++row) {
            const F &Ac = A6[comp[row][col]];
            out[row] += (gfac[0] * Ac(i + di, j + dj, k + dk) - gfac[1] * Ac(i - di, j - dj, k - dk)) * inv2h;
        }
    }
    out[0] *= 2.0;
    out[1] *= 2.0;
    out[2] *= 2.0;
}

__device__ __forceinline__ void shift_source_point(const double *__restrict__ psi, const double *__restrict__ xi,
                                                   const double *const *A6, int i, int j, int k, int n, double h,
                                                   double a, double c, double (&out)[3])
{
    const PeriodicField A[6] = {{A6[0], n}, {A6[1], n}, {A6[2], n}, {A6[3], n}, {A6[4], n}, {A6[5], n}};
    shift_source_f(PeriodicField{psi, n}, PeriodicField{xi, n}, A, i, j, k, h, a, c, out);
}

} // namespace detail
} // namespace grmg
