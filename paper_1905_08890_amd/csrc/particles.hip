// Particle evolution with the solved metric (paper sec. 4.4, and the leapfrog
// of the appendix on time evolution): the kick, split into five ordered
// substeps over the force contributions, and the drift with the coordinate
// velocity.  One thread per particle; the metric quantities at a particle are
// the cloud-in-cell interpolation (the deposit's cell-centred weights and
// periodic wrap) of the grid values and of their 3-point central-difference
// gradients, evaluated at the eight cloud corners from the grid arrays.
#include <cmath>

#include "gr_internal.h"

namespace grmg {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct PField {
    double Phi, Psi, beta[3];
    double dPhi[3], dPsi[3];
    double dbeta[3][3]; // dbeta[i][j] = d_i beta^j
};

struct Metric {
    const double *Phi, *Psi, *beta[3];
    int n;
    double inv2h;
};

// central difference d_dir g at cell (i, j, k) (wrapped indices)
__device__ __forceinline__ double dc(const double *__restrict__ g, int dir, int i, int j, int k, int n, double inv2h)
{
    const long plane = (long)n * n;
    long pp, pm;
    if (dir == 0) {
        pp = k * plane + (long)j * n + wrapc(i + 1, n);
        pm = k * plane + (long)j * n + wrapc(i - 1, n);
    } else if (dir == 1) {
        pp = k * plane + (long)wrapc(j + 1, n) * n + i;
        pm = k * plane + (long)wrapc(j - 1, n) * n + i;
    } else {
        pp = wrapc(k + 1, n) * plane + (long)j * n + i;
        pm = wrapc(k - 1, n) * plane + (long)j * n + i;
    }
    return (g[pp] - g[pm]) * inv2h;
}

template <bool GRAD>
__device__ void particle_fields(const Metric &M, const double *x, PField &F)
{
    const int n = M.n;
    const double inv_h = (double)n;
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        const double g = x[d] * inv_h - 0.5;
        const double fl = floor(g);
        i0[d] = (int)fl;
        t[d] = g - fl;
    }
    F = PField{};
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        const double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        const int ci = wrapc(i0[0] + ox, n), cj = wrapc(i0[1] + oy, n), ck = wrapc(i0[2] + oz, n);
        const long p = ((long)ck * n + cj) * n + ci;
        F.Phi += w * M.Phi[p];
        F.Psi += w * M.Psi[p];
        for (int d = 0; d < 3; ++d) F.beta[d] += w * M.beta[d][p];
        if (GRAD)
            for (int d = 0; d < 3; ++d) {
                F.dPhi[d] += w * dc(M.Phi, d, ci, cj, ck, n, M.inv2h);
                F.dPsi[d] += w * dc(M.Psi, d, ci, cj, ck, n, M.inv2h);
                for (int j = 0; j < 3; ++j) F.dbeta[d][j] += w * dc(M.beta[j], d, ci, cj, ck, n, M.inv2h);
            }
    }
}

__device__ __forceinline__ double lorentz_W(double a, double c, double Psi, const double u[3])
{
    const double chi = 1.0 - Psi / (2.0 * a * a * c * c);
    const double chi2 = chi * chi;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return sqrt(c * c + uu / (a * a * chi2 * chi2));
}

// Five substeps of u_i += dt c_j (f_j)_i (see gr_kick); c_j from the velocity
// as updated by the substeps before it.
__global__ void __launch_bounds__(TPB) k_kick(Metric M, double a, double c, const double *__restrict__ pos,
                                              double *__restrict__ u, long np, double dt, int order)
{
    const long q = (long)blockIdx.x * TPB + threadIdx.x;
    if (q >= np) return;
    PField F;
    const double x[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
    particle_fields<true>(M, x, F);
    double uq[3] = {u[3 * q], u[3 * q + 1], u[3 * q + 2]};
    for (int s = 0; s < 5; ++s) {
        const int j = order == GR_KICK_FORWARD ? s + 1 : 5 - s;
        double cj, f[3];
        if (j <= 3) {
            cj = -uq[j - 1];
            for (int i = 0; i < 3; ++i) f[i] = -F.dbeta[i][j - 1];
        } else {
            const double W = lorentz_W(a, c, F.Psi, uq);
            if (j == 4) {
                cj = (W * W - c * c) / (W * c) * (1.0 + F.Phi / (a * a * c * c)) / (1.0 - F.Psi / (2.0 * a * a * c * c));
                for (int i = 0; i < 3; ++i) f[i] = -F.dPsi[i];
            } else {
                cj = W / c;
                for (int i = 0; i < 3; ++i) f[i] = -F.dPhi[i];
            }
        }
        for (int i = 0; i < 3; ++i) uq[i] += dt * cj * f[i];
    }
    for (int i = 0; i < 3; ++i) u[3 * q + i] = uq[i];
}

// x^i += dt V^i with the fields at the old position, wrapped into [0, 1)
__global__ void __launch_bounds__(TPB) k_drift(Metric M, double a, double c, double *__restrict__ pos,
                                               const double *__restrict__ u, long np, double dt)
{
    const long q = (long)blockIdx.x * TPB + threadIdx.x;
    if (q >= np) return;
    PField F;
    double x[3] = {pos[3 * q], pos[3 * q + 1], pos[3 * q + 2]};
    particle_fields<false>(M, x, F);
    const double uq[3] = {u[3 * q], u[3 * q + 1], u[3 * q + 2]};
    const double W = lorentz_W(a, c, F.Psi, uq);
    const double chi = 1.0 - F.Psi / (2.0 * a * a * c * c);
    const double chi2 = chi * chi;
    const double fac = (1.0 + F.Phi / (a * a * c * c)) / (chi2 * chi2) * (c / W);
    for (int d = 0; d < 3; ++d) {
        const double v = fac * uq[d] - F.beta[d];
        double y = x[d] + dt * v;
        y -= floor(y);
        if (y >= 1.0) y = 0.0;
        pos[3 * q + d] = y;
    }
}

// Newtonian kick of the temporary synchronisation: u_i -= dt d_i Phi_N (CIC
// interpolation of the central difference at the eight cloud corners)
__global__ void __launch_bounds__(TPB) k_newton_kick(const double *__restrict__ phiN, int n, double inv2h,
                                                     const double *__restrict__ pos, double *__restrict__ u, long np,
                                                     double dt)
{
    const long q = (long)blockIdx.x * TPB + threadIdx.x;
    if (q >= np) return;
    int i0[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        const double g = pos[3 * q + d] * (double)n - 0.5;
        const double fl = floor(g);
        i0[d] = (int)fl;
        t[d] = g - fl;
    }
    double grad[3] = {0.0, 0.0, 0.0};
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        const double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        const int ci = wrapc(i0[0] + ox, n), cj = wrapc(i0[1] + oy, n), ck = wrapc(i0[2] + oz, n);
        for (int d = 0; d < 3; ++d) grad[d] += w * dc(phiN, d, ci, cj, ck, n, inv2h);
    }
    for (int d = 0; d < 3; ++d) u[3 * q + d] -= dt * grad[d];
}

} // namespace

void launch_newton_kick(hipStream_t s, int n, const double *phiN, const double *pos, double *u, long np, double dt)
{
    if (np <= 0) return;
    k_newton_kick<<<(unsigned)((np + TPB - 1) / TPB), TPB, 0, s>>>(phiN, n, 0.5 * n, pos, u, np, dt);
}

void launch_kick(hipStream_t s, int n, double a, double c, const double *Phi, const double *Psi,
                 const double *const beta[3], const double *pos, double *u, long np, double dt, int order)
{
    if (np <= 0) return;
    const Metric M{Phi, Psi, {beta[0], beta[1], beta[2]}, n, 0.5 * n};
    k_kick<<<(unsigned)((np + TPB - 1) / TPB), TPB, 0, s>>>(M, a, c, pos, u, np, dt, order);
}

void launch_drift(hipStream_t s, int n, double a, double c, const double *Phi, const double *Psi,
                  const double *const beta[3], double *pos, const double *u, long np, double dt)
{
    if (np <= 0) return;
    const Metric M{Phi, Psi, {beta[0], beta[1], beta[2]}, n, 0.5 * n};
    k_drift<<<(unsigned)((np + TPB - 1) / TPB), TPB, 0, s>>>(M, a, c, pos, u, np, dt);
}

} // namespace grmg
