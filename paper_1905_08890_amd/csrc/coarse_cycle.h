// The coarse levels of a V-cycle run by one workgroup (device code shared by
// the single-grid kernels and the batched ones).  Included inside namespace
// grmg::detail after stencil_ops.h.
#pragma once

#include "stencil_ops.h"

namespace grmg {
namespace detail {

// The V-cycle below (and including) level ls, run by one workgroup: every
// level is small enough to live in L2, so one launch with block barriers
// replaces the ~10 launches per level of the multi-kernel path.  Same steps,
// same order: nu1 sweeps, residual + restriction, coarse source, ..., 32
// sweeps and mean projection at the coarsest, prolongation, nu2 sweeps.
// FAS kinds: phi0 = R phi, f^H = L^H(R phi) - R eps.  Linearised kinds
// (correction scheme): b^H = R(b - J e), e^H = 0.
constexpr int kCoarseThreads = 1024;

template <int KIND, typename T>
__device__ void cv_sweep(T *__restrict__ phi, const T *__restrict__ f, const T *__restrict__ c1,
                         const T *__restrict__ c2, int n, T inv_h2, OpConst oc, T Fb, T fs)
{
    const int half = n >> 1, tot = n * n * half;
    const SmallDiv dh(half), dn(n);
    const T rJ = poisson_inv_diag(inv_h2);
    for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < tot; t += kCoarseThreads) {
            const int r = dh.div(t), z = dn.div(r);
            const int x2 = t - r * half, y = r - z * n;
            const int i = 2 * x2 + ((y + z + colour) & 1);
            const long p = lin(i, y, z, n);
            const T ph = phi[p];
            T J;
            const T L = op_point<KIND, T>(ph, nb_sum(phi, i, y, z, n), inv_h2, load_c1<KIND>(c1, p),
                                          load_c2<KIND>(c2, p), oc, Fb, J);
            phi[p] = newton_update<KIND, T>(ph, L, f[p] - fs, J, rJ);
        }
        __syncthreads();
    }
}

__device__ double cv_block_sum(double v)
{
    __shared__ double sh[kCoarseThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kCoarseThreads / 64; ++w) s += sh[w];
    __syncthreads();
    return s; // every thread gets the same fixed-order sum
}

template <int KIND, typename T>
__device__ void coarse_vcycle_body(const CoarseLevelsT<T> &C, int nu1, int nu2, OpConst oc, const T Fb0,
                                   const T fs0) // frozen scalars of C's first level (zero unless the finest)
{
    constexpr bool LIN = KIND >= K_LIN_POISSON;
    const int L = C.nl;
    for (int i = 0; i < L - 1; ++i) {
        const int n = C.n[i], m = n >> 1;
        const T inv_h2 = T(C.inv_h2[i]);
        const T Fb = i == 0 ? Fb0 : T(0), fs = i == 0 ? fs0 : T(0);
        for (int it = 0; it < nu1; ++it) cv_sweep<KIND, T>(C.phi[i], C.f[i], C.c1[i], C.c2[i], n, inv_h2, oc, Fb, fs);
        const int M = m * m * m;
        const SmallDiv dm(m);
        for (int q = threadIdx.x; q < M; q += kCoarseThreads) {
            const int r = dm.div(q), Z = dm.div(r);
            const int X = q - r * m, Y = r - Z * m;
            T sr = 0, sp = 0;
            for (int c = 0; c < 8; ++c) {
                const int a = 2 * X + (c & 1), b = 2 * Y + ((c >> 1) & 1), d = 2 * Z + (c >> 2);
                const long p = lin(a, b, d, n);
                const T ph = C.phi[i][p];
                T Jd;
                const T Lv = op_point<KIND, T>(ph, nb_sum(C.phi[i], a, b, d, n), inv_h2, load_c1<KIND>(C.c1[i], p),
                                               load_c2<KIND>(C.c2[i], p), oc, Fb, Jd);
                sr += Lv - (C.f[i][p] - fs);
                sp += ph;
            }
            if constexpr (LIN) {
                C.f[i + 1][q] = -sr / T(8);
                C.phi[i + 1][q] = T(0);
            } else {
                const T rp = sp / T(8);
                C.phi[i + 1][q] = rp;
                C.phi0[i + 1][q] = rp;
                C.tmp[i + 1][q] = sr / T(8);
            }
        }
        __syncthreads();
        if constexpr (!LIN) {
            const T inv_H2 = T(C.inv_h2[i + 1]);
            for (int q = threadIdx.x; q < M; q += kCoarseThreads) {
                const int r = dm.div(q), Z = dm.div(r);
                const int X = q - r * m, Y = r - Z * m;
                T Jd;
                const T Lv = op_point<KIND, T>(C.phi[i + 1][q], nb_sum(C.phi[i + 1], X, Y, Z, m), inv_H2,
                                               load_c1<KIND>(C.c1[i + 1], q), load_c2<KIND>(C.c2[i + 1], q), oc, T(0),
                                               Jd);
                C.f[i + 1][q] = Lv - C.tmp[i + 1][q];
            }
            __syncthreads();
        }
    }
    if (C.n[L - 1] * C.n[L - 1] * C.n[L - 1] <= 64) {
        // coarsest level of at most 64 points: one wavefront, one point per lane,
        // neighbours by lane shuffles (no block barriers between the sweeps)
        const int i = L - 1, n = C.n[i], N = n * n * n;
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            const bool on = lane < N;
            const int a = lane % n, b = (lane / n) % n, d = lane / (n * n);
            const int xp = (int)lin(wrapi(a + 1, n), b, d, n), xm = (int)lin(wrapi(a - 1, n), b, d, n);
            const int yp = (int)lin(a, wrapi(b + 1, n), d, n), ym = (int)lin(a, wrapi(b - 1, n), d, n);
            const int zp = (int)lin(a, b, wrapi(d + 1, n), n), zm = (int)lin(a, b, wrapi(d - 1, n), n);
            const T inv_h2 = T(C.inv_h2[i]);
            const T Fb = i == 0 ? Fb0 : T(0), fs = i == 0 ? fs0 : T(0);
            T ph = on ? C.phi[i][lane] : T(0);
            const T fv = on ? C.f[i][lane] : T(0);
            const T cv1 = on ? load_c1<KIND>(C.c1[i], lane) : T(0);
            const T cv2 = on ? load_c2<KIND>(C.c2[i], lane) : T(0);
            const T old = ph;
            const int par = (a + b + d) & 1;
            for (int it = 0; it < kCoarseSweeps; ++it)
                for (int colour = 0; colour < 2; ++colour) {
                    const T nbs = __shfl(ph, on ? xp : lane, 64) + __shfl(ph, on ? xm : lane, 64) +
                                  __shfl(ph, on ? yp : lane, 64) + __shfl(ph, on ? ym : lane, 64) +
                                  __shfl(ph, on ? zp : lane, 64) + __shfl(ph, on ? zm : lane, 64);
                    if (on && par == colour) {
                        T J;
                        const T Lv = op_point<KIND, T>(ph, nbs, inv_h2, cv1, cv2, oc, Fb, J);
                        ph = newton_update<KIND, T>(ph, Lv, fv - fs, J, poisson_inv_diag(inv_h2));
                    }
                }
            double dsum = on ? (double)(ph - old) : 0.0;
            for (int off = 1; off < 64; off <<= 1) dsum += __shfl_xor(dsum, off, 64);
            ph -= T(dsum / (double)N);
            if (on) C.phi[i][lane] = ph;
        }
        __syncthreads();
    } else { // coarsest: sweeps, then remove the mean of the correction
        const int i = L - 1, n = C.n[i], N = n * n * n;
        const T inv_h2 = T(C.inv_h2[i]);
        const T Fb = i == 0 ? Fb0 : T(0), fs = i == 0 ? fs0 : T(0);
        for (int q = threadIdx.x; q < N; q += kCoarseThreads) C.tmp[i][q] = C.phi[i][q];
        __syncthreads();
        for (int it = 0; it < kCoarseSweeps; ++it)
            cv_sweep<KIND, T>(C.phi[i], C.f[i], C.c1[i], C.c2[i], n, inv_h2, oc, Fb, fs);
        double d = 0.0;
        for (int q = threadIdx.x; q < N; q += kCoarseThreads) d += (double)(C.phi[i][q] - C.tmp[i][q]);
        const T mean = T(cv_block_sum(d) / (double)N);
        for (int q = threadIdx.x; q < N; q += kCoarseThreads) C.phi[i][q] -= mean;
        __syncthreads();
    }
    for (int i = L - 2; i >= 0; --i) {
        const int n = C.n[i], m = n >> 1, N = n * n * n;
        const T inv_h2 = T(C.inv_h2[i]);
        const T Fb = i == 0 ? Fb0 : T(0), fs = i == 0 ? fs0 : T(0);
        const SmallDiv dn(n);
        for (int p = threadIdx.x; p < N; p += kCoarseThreads) {
            const int r = dn.div(p), d = dn.div(r);
            const int a = p - r * n, b = r - d * n;
            const int I = a >> 1, J = b >> 1, K = d >> 1;
            const int Is[2] = {I, wrapi(I + ((a & 1) ? 1 : -1), m)};
            const int Js[2] = {J, wrapi(J + ((b & 1) ? 1 : -1), m)};
            const int Ks[2] = {K, wrapi(K + ((d & 1) ? 1 : -1), m)};
            T v = 0;
            for (int c = 0; c < 8; ++c) {
                const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                const T w = (ox ? T(0.25) : T(0.75)) * (oy ? T(0.25) : T(0.75)) * (oz ? T(0.25) : T(0.75));
                const long q = lin(Is[ox], Js[oy], Ks[oz], m);
                v += w * (LIN ? C.phi[i + 1][q] : C.phi[i + 1][q] - C.phi0[i + 1][q]);
            }
            C.phi[i][p] += v;
        }
        __syncthreads();
        for (int it = 0; it < nu2; ++it) cv_sweep<KIND, T>(C.phi[i], C.f[i], C.c1[i], C.c2[i], n, inv_h2, oc, Fb, fs);
    }
}

// The same cycle with every level held in LDS (levels up to 16^3 fit): the
// first level's iterate, source and all levels' coefficients are copied in,
// the first level's iterate is copied back; barriers then cost LDS latency
// instead of L2 round trips.  TG is the type of the arrays in global memory,
// TC the type the cycle computes in (FP64 also for the FP32 correction
// cycles: their coarsest levels and mean constraint are solved in FP64).
constexpr size_t kCoarseLdsBytes = 150 * 1024;

template <int KIND, typename TG, typename T>
__host__ __device__ size_t coarse_lds_layout(const CoarseLevelsT<TG> &G, CoarseLevelsT<T> *S, T *base)
{
    constexpr bool LIN = KIND >= K_LIN_POISSON;
    constexpr int NC = kNumCoef<KIND>();
    size_t off = 0;
    auto take = [&](long count) -> T * {
        T *p = base ? base + off : nullptr;
        off += (size_t)count;
        return p;
    };
    for (int i = 0; i < G.nl; ++i) {
        const long N = (long)G.n[i] * G.n[i] * G.n[i];
        T *phi = take(N);
        T *phi0 = (i >= 1 && !LIN) ? take(N) : nullptr;
        T *f = take(N);
        T *c1 = NC >= 1 ? take(N) : nullptr;
        T *c2 = NC >= 2 ? take(N) : nullptr;
        T *tmp = (i >= 1 || G.nl == 1) ? take(N) : nullptr;
        if (S) {
            S->n[i] = G.n[i];
            S->inv_h2[i] = G.inv_h2[i];
            S->phi[i] = phi;
            S->phi0[i] = phi0;
            S->f[i] = f;
            S->c1[i] = c1;
            S->c2[i] = c2;
            S->tmp[i] = tmp;
        }
    }
    if (S) S->nl = G.nl;
    return off * sizeof(T);
}

template <int KIND, typename TG, typename T>
__device__ void coarse_cycle_lds(const CoarseLevelsT<TG> &G, int nu1, int nu2, OpConst oc,
                                 const double *__restrict__ fbar0, const double *__restrict__ fshift0)
{
    constexpr int NC = kNumCoef<KIND>();
    __shared__ T lds[kCoarseLdsBytes / sizeof(T)];
    __shared__ CoarseLevelsT<T> S; // level table, read by every thread (kept out of private memory)
    if (threadIdx.x == 0) coarse_lds_layout<KIND, TG, T>(G, &S, lds);
    __syncthreads();
    const long N0 = (long)G.n[0] * G.n[0] * G.n[0];
    for (long q = threadIdx.x; q < N0; q += kCoarseThreads) {
        S.phi[0][q] = T(G.phi[0][q]);
        S.f[0][q] = T(G.f[0][q]);
    }
    for (int i = 0; i < G.nl; ++i) {
        const long N = (long)G.n[i] * G.n[i] * G.n[i];
        for (long q = threadIdx.x; q < N; q += kCoarseThreads) {
            if (NC >= 1) S.c1[i][q] = T(G.c1[i][q]);
            if (NC >= 2) S.c2[i][q] = T(G.c2[i][q]);
        }
    }
    __syncthreads();
    coarse_vcycle_body<KIND, T>(S, nu1, nu2, oc, T(*fbar0), T(*fshift0));
    __syncthreads();
    for (long q = threadIdx.x; q < N0; q += kCoarseThreads) G.phi[0][q] = TG(S.phi[0][q]);
}

} // namespace detail
} // namespace grmg
