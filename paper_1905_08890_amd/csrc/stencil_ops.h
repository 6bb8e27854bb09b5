// Per-point device arithmetic of the multigrid operators, shared by the
// single-grid and batched kernels (included inside namespace grmg::detail).
#pragma once

#include "gr_internal.h"

namespace grmg {
namespace detail {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ long lin(int i, int j, int k, int n) { return ((long)k * n + j) * n + i; }

// Sum of the six face neighbours of (i,j,k) with periodic wrap, added as
// x-, x+, y-, y+, z-, z+: the order of the LDS-tiled sweeps and residuals, so
// every smoother launch shape rounds alike.
template <typename T>
__device__ __forceinline__ T nb_sum(const T *__restrict__ p, int i, int j, int k, int n)
{
    int ip = wrapi(i + 1, n), im = wrapi(i - 1, n);
    int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
    int kp = wrapi(k + 1, n), km = wrapi(k - 1, n);
    return p[lin(im, j, k, n)] + p[lin(ip, j, k, n)] + p[lin(i, jm, k, n)] + p[lin(i, jp, k, n)]
         + p[lin(i, j, km, n)] + p[lin(i, j, kp, n)];
}

// number of coefficient arrays an operator reads
template <int KIND> constexpr int kNumCoef()
{
    return (KIND == GR_KIND_POISSON || KIND == K_LIN_POISSON) ? 0 : (KIND == K_LIN_HAM ? 2 : 1);
}

// L(phi) at a point (without the source) and dL/dphi there.
// c1: AA (Hamiltonian), m2 (CMC), c (linearised kinds); c2: a (linearised Hamiltonian).
template <int KIND, typename T>
__device__ __forceinline__ T op_point(T ph, T nbs, T inv_h2, T c1, T c2, OpConst oc, T Fbar, T &J)
{
    const T lap = (nbs - T(6) * ph) * inv_h2;
    if constexpr (KIND == GR_KIND_POISSON || KIND == K_LIN_POISSON) {
        J = T(-6) * inv_h2;
        return lap;
    } else if constexpr (KIND == GR_KIND_CMC) {
        J = T(-6) * inv_h2 - c1;
        return lap - c1 * ph;
    } else if constexpr (KIND == K_LIN_CMC) {
        J = T(-6) * inv_h2 + c1;
        return lap + c1 * ph;
    } else if constexpr (KIND == K_LIN_HAM) {
        J = T(-6) * c2 * inv_h2 + c1;
        return c2 * lap + c1 * ph;
    } else {
        const double kap = oc.kappa, A = oc.A;
        const double chi = 1.0 - kap * ph;
        const double chi2 = chi * chi;
        const double chi5 = chi2 * chi2 * chi;
        const double chi6 = chi5 * chi;
        // one FP64 division per point: negative powers from 1/chi by products
        const double r = 1.0 / chi;
        const double r2 = r * r;
        const double chim6 = r2 * r2 * r2;
        const double chim7 = chim6 * r;
        J = -kap * lap - 6.0 * chi * inv_h2 - 6.0 * A * kap * chi5 - 1.5 * kap * c1 * chim7 - kap * Fbar;
        return chi * lap + A * (chi6 - 1.0) - 0.25 * c1 * chim6 + Fbar * chi;
    }
}

// The point update ph - (L - fe) / J of every smoother.  The correction
// equation of the Poisson kind (FP32 sweeps, FP64 coarse levels) has the constant
// diagonal J = -6/h^2: there the update multiplies by its reciprocal rJ (formed
// once per kernel from inv_h2), within an ulp of the division, which the
// correction does not need.
template <typename T> __device__ __forceinline__ T poisson_inv_diag(T inv_h2) { return T(1) / (T(-6) * inv_h2); }

template <int KIND, typename T>
__device__ __forceinline__ T newton_update(T ph, T L, T fe, T J, T rJ)
{
    if constexpr (KIND == K_LIN_POISSON)
        return ph - (L - fe) * rJ;
    else
        return ph - (L - fe) / J;
}

// t / d for 0 <= t < 2^24: for 1 < d < 2^8 a multiply-high with m = ceil(2^32 / d)
// (the error term t (m d - 2^32) < 2^24 2^8 keeps the quotient exact), else a division.
struct SmallDiv {
    unsigned m;
    int d;
    __device__ __forceinline__ explicit SmallDiv(int d_)
        : m(d_ > 1 && d_ < 256 ? 0xffffffffu / (unsigned)d_ + 1u : 0u), d(d_)
    {
    }
    __device__ __forceinline__ int div(int t) const { return m ? (int)__umulhi((unsigned)t, m) : t / d; }
};

template <int KIND, typename T>
__device__ __forceinline__ T load_c1(const T *__restrict__ c1, long p)
{
    return kNumCoef<KIND>() >= 1 ? c1[p] : T(0);
}
template <int KIND, typename T>
__device__ __forceinline__ T load_c2(const T *__restrict__ c2, long p)
{
    return kNumCoef<KIND>() >= 2 ? c2[p] : T(0);
}

} // namespace detail
} // namespace grmg
