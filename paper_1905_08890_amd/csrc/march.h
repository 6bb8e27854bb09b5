// Plane-marching residual kernels: one tile x z-chunk as a device function
// (shared by the single-grid kernels and the batched kernels).
#pragma once

#include <type_traits>

#include "stencil_ops.h"

namespace grmg {
namespace detail {

// A workgroup of 32 x 8 threads owns one (x, y) point each of a 32 x 8 tile
// and marches a chunk of zc planes in z.  Each plane of the iterate, with a
// 1-cell halo ring, goes to one of two LDS buffers (one barrier per plane);
// the z-neighbours stay in registers.  All reads of a plane are issued two
// planes ahead, in two alternating register sets.  Per point the iterate is
// read once from memory (plus the halo ring, mostly from L2), the source and
// coefficients once.  Modes:
//   M_NORMS        sums of eps^2 and (f - fshift)^2 (stopping test)
//   M_IR           as M_NORMS, plus the FP32 correction source b = -eps and,
//                  for the Hamiltonian, a = chi and c = dL/dPsi + 6 chi/h^2
//   M_RESTRICT     FAS: R eps, R phi (also as phi0) on the coarse level
//   M_RESTRICT_LIN correction scheme: R(b - J e) and a zero coarse e
//   M_IRU          Poisson refinement step: the iterate read is phi + e (the
//                  FP32 correction, e32), written to o1 (out of place), then
//                  as M_IR for that updated iterate
// The restriction modes sum z pairs in registers and x / y pairs across lanes.
enum { M_NORMS = 0, M_IR = 1, M_RESTRICT = 2, M_RESTRICT_LIN = 3, M_IRU = 4 };
constexpr int MTX = 32, MTY = 8, MNT = MTX * MTY;
constexpr int MHALO = 2 * (MTX + 2) + 2 * MTY; // halo ring of a plane

// One workgroup's tile (x0, y0) and z-chunk [z0, z0 + zc); norm[0..1] get this
// thread's sums of eps^2 and (f - fshift)^2 (norm modes).
template <int MODE, int KIND, typename T>
__device__ __forceinline__ void march_tile(const T *__restrict__ phi, const T *__restrict__ f,
                                           const T *__restrict__ c1, const T *__restrict__ c2, const int n,
                                           const int zc, const T inv_h2, OpConst oc, const T Fb, const T fs,
                                           const int x0, const int y0, const int z0, T *__restrict__ o1,
                                           T *__restrict__ o2, T *__restrict__ o3, float *__restrict__ b32,
                                           float *__restrict__ a32, float *__restrict__ c32, double *norm,
                                           const float *__restrict__ e32 = nullptr)
{
    constexpr int FW = MTX + 2, FH = MTY + 2;
    constexpr int NC = kNumCoef<KIND>();
    __shared__ T buf[2][FH * FW];
    const int tid = threadIdx.x;
    const int tx = tid % MTX, ty = tid / MTX;
    const long plane = (long)n * n;
    const long own = (long)(y0 + ty) * n + x0 + tx;
    // halo ring position of this thread (tid < MHALO): frame row / column
    int hr = 0, hc = 0;
    if (tid < 2 * (MTX + 2)) {
        hr = tid < MTX + 2 ? 0 : FH - 1;
        hc = tid < MTX + 2 ? tid : tid - (MTX + 2);
    } else if (tid < MHALO) {
        const int k = tid - 2 * (MTX + 2);
        hr = 1 + k / 2;
        hc = (k & 1) ? FW - 1 : 0;
    }
    const long hoff = (long)wrapi(y0 + hr - 1, n) * n + wrapi(x0 + hc - 1, n);
    const int fo = (ty + 1) * FW + tx + 1; // own frame index

    struct Set {
        T own, halo, f, c, a;
    };
    // the iterate at a point (M_IRU: updated by the correction on the fly)
    auto it_at = [&](long q) { return MODE == M_IRU ? phi[q] + T(e32[q]) : phi[q]; };
    auto load = [&](Set &S, int z) {
        const long zo = (long)wrapi(z, n) * plane;
        S.own = it_at(zo + own);
        if (tid < MHALO) S.halo = it_at(zo + hoff);
        S.f = f[zo + own];
        if (NC >= 1) S.c = c1[zo + own];
        if (NC >= 2) S.a = c2[zo + own];
    };
    Set A, B;
    A.own = A.halo = A.f = A.c = A.a = T(0);
    B = A;
    T below = it_at((long)wrapi(z0 - 1, n) * plane + own);
    load(A, z0);
    load(B, z0 + 1);
    double v0 = 0.0, v1 = 0.0; // norm sums
    T sr = 0, sp = 0;          // restriction sums over a z pair

    auto body = [&](const int z, Set &S, const Set &Nx) {
        T *pl = buf[z & 1];
        pl[fo] = S.own;
        if (tid < MHALO) pl[hr * FW + hc] = S.halo;
        __syncthreads();
        const T ph = S.own;
        const T nbs = pl[fo - 1] + pl[fo + 1] + pl[fo - FW] + pl[fo + FW] + below + Nx.own;
        T J;
        const T L = op_point<KIND, T>(ph, nbs, inv_h2, S.c, S.a, oc, Fb, J);
        const long p = (long)z * plane + own;
        if constexpr (MODE == M_NORMS || MODE == M_IR || MODE == M_IRU) {
            const double fe = (double)S.f - (double)fs;
            const double e = (double)L - fe;
            v0 += e * e;
            v1 += fe * fe;
            if constexpr (MODE == M_IRU) {
                o1[p] = ph;
                b32[p] = (float)(-e);
            }
            if constexpr (MODE == M_IR) {
                b32[p] = (float)(-e);
                if constexpr (KIND == GR_KIND_HAMILTONIAN) {
                    const double chi = 1.0 - oc.kappa * (double)ph;
                    a32[p] = (float)chi;
                    c32[p] = (float)((double)J + 6.0 * chi * (double)inv_h2);
                }
            }
        } else {
            sr += (MODE == M_RESTRICT) ? L - (S.f - fs) : S.f - L;
            sp += ph;
            if (z & 1) { // a z pair is complete: add the x and y pairs across lanes
                T r2 = sr + __shfl_xor(sr, 1, 64);
                T p2 = sp + __shfl_xor(sp, 1, 64);
                r2 += __shfl_xor(r2, 32, 64);
                p2 += __shfl_xor(p2, 32, 64);
                if (((tx | ty) & 1) == 0) {
                    const int m = n >> 1;
                    const long q = ((long)(z >> 1) * m + ((y0 + ty) >> 1)) * m + ((x0 + tx) >> 1);
                    if constexpr (MODE == M_RESTRICT) {
                        o1[q] = p2 / T(8); // R phi
                        o2[q] = p2 / T(8); // phi0
                        o3[q] = r2 / T(8); // R eps
                    } else {
                        o1[q] = r2 / T(8); // coarse b
                        o2[q] = T(0);      // coarse e
                    }
                }
                sr = 0;
                sp = 0;
            }
        }
        below = ph;
        if (z + 2 < z0 + zc) load(S, z + 2);
        else if (z + 2 == z0 + zc) S.own = it_at((long)wrapi(z + 2, n) * plane + own); // last plane's z + 1
    };
    for (int z = z0; z < z0 + zc; z += 2) {
        body(z, A, B);
        body(z + 1, B, A);
    }
    norm[0] = v0;
    norm[1] = v1;
}

// The same plane march on 64 x 8 tiles with 256 threads, each owning an
// x-pair (2 tx, 2 tx + 1) of one row: the iterate, source and coefficients
// arrive as 16-byte (FP64) or 8-byte (FP32) pair loads, so every thread keeps
// twice the bytes in flight per load instruction.  Per point the arithmetic,
// the neighbour order and the restriction's pairing are those of march_tile
// (the x-pair of a restriction cell now sits in one thread), so the per-point
// outputs are bit-identical; only the norm sums are added in another order.
constexpr int M2TX = 64, M2TY = 8, M2NT = (M2TX / 2) * M2TY;
constexpr int M2HALO = 2 * (M2TX + 2) + 2 * M2TY;

template <int MODE, int KIND, typename T>
__device__ __forceinline__ void march_tile2(const T *__restrict__ phi, const T *__restrict__ f,
                                            const T *__restrict__ c1, const T *__restrict__ c2, const int n,
                                            const int zc, const T inv_h2, OpConst oc, const T Fb, const T fs,
                                            const int x0, const int y0, const int z0, T *__restrict__ o1,
                                            T *__restrict__ o2, T *__restrict__ o3, float *__restrict__ b32,
                                            float *__restrict__ a32, float *__restrict__ c32, double *norm,
                                            const float *__restrict__ e32 = nullptr)
{
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    constexpr int FW = M2TX + 2, FH = M2TY + 2;
    constexpr int NC = kNumCoef<KIND>();
    __shared__ T buf[2][FH * FW];
    const int tid = threadIdx.x;
    const int tx = tid % (M2TX / 2), ty = tid / (M2TX / 2);
    const long plane = (long)n * n;
    const long own = (long)(y0 + ty) * n + x0 + 2 * tx; // even point of the pair
    int hr = 0, hc = 0;
    if (tid < 2 * FW) {
        hr = tid < FW ? 0 : FH - 1;
        hc = tid < FW ? tid : tid - FW;
    } else if (tid < M2HALO) {
        const int k = tid - 2 * FW;
        hr = 1 + k / 2;
        hc = (k & 1) ? FW - 1 : 0;
    }
    const long hoff = (long)wrapi(y0 + hr - 1, n) * n + wrapi(x0 + hc - 1, n);
    const int fo = (ty + 1) * FW + 2 * tx + 1; // frame index of the even point

    auto ld2 = [](const T *p) { return *reinterpret_cast<const T2 *>(p); };
    auto it2 = [&](long q) {
        T2 v = ld2(phi + q);
        if constexpr (MODE == M_IRU) {
            const float2 e = *reinterpret_cast<const float2 *>(e32 + q);
            v.x = v.x + T(e.x);
            v.y = v.y + T(e.y);
        }
        return v;
    };
    auto it1 = [&](long q) { return MODE == M_IRU ? phi[q] + T(e32[q]) : phi[q]; };
    struct Set {
        T2 own, f, c, a;
        T halo;
    };
    auto load = [&](Set &S, int z) {
        const long zo = (long)wrapi(z, n) * plane;
        S.own = it2(zo + own);
        if (tid < M2HALO) S.halo = it1(zo + hoff);
        S.f = ld2(f + zo + own);
        if (NC >= 1) S.c = ld2(c1 + zo + own);
        if (NC >= 2) S.a = ld2(c2 + zo + own);
    };
    Set A, B;
    A.own = A.f = A.c = A.a = T2{T(0), T(0)};
    A.halo = T(0);
    B = A;
    T2 below = it2((long)wrapi(z0 - 1, n) * plane + own);
    load(A, z0);
    load(B, z0 + 1);
    double v0 = 0.0, v1 = 0.0;           // norm sums
    T sr[2] = {0, 0}, sp[2] = {0, 0};    // restriction sums over a z pair, per point

    auto body = [&](const int z, Set &S, const Set &Nx) {
        T *pl = buf[z & 1];
        pl[fo] = S.own.x;
        pl[fo + 1] = S.own.y;
        if (tid < M2HALO) pl[hr * FW + hc] = S.halo;
        __syncthreads();
        const T own_v[2] = {S.own.x, S.own.y};
        const T bel[2] = {below.x, below.y};
        const T abv[2] = {Nx.own.x, Nx.own.y};
        const T cc[2] = {S.c.x, S.c.y}, aa[2] = {S.a.x, S.a.y}, ff[2] = {S.f.x, S.f.y};
        T Lv[2], Jv[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int q = fo + j;
            const T nbs = pl[q - 1] + pl[q + 1] + pl[q - FW] + pl[q + FW] + bel[j] + abv[j];
            Lv[j] = op_point<KIND, T>(own_v[j], nbs, inv_h2, cc[j], aa[j], oc, Fb, Jv[j]);
        }
        const long p = (long)z * plane + own;
        if constexpr (MODE == M_NORMS || MODE == M_IR || MODE == M_IRU) {
            float bv[2], av[2], cv[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const double fe = (double)ff[j] - (double)fs;
                const double e = (double)Lv[j] - fe;
                v0 += e * e;
                v1 += fe * fe;
                bv[j] = (float)(-e);
                if constexpr (KIND == GR_KIND_HAMILTONIAN) {
                    const double chi = 1.0 - oc.kappa * (double)own_v[j];
                    av[j] = (float)chi;
                    cv[j] = (float)((double)Jv[j] + 6.0 * chi * (double)inv_h2);
                }
            }
            if constexpr (MODE == M_IRU) *reinterpret_cast<T2 *>(o1 + p) = S.own;
            if constexpr (MODE == M_IR || MODE == M_IRU) *reinterpret_cast<float2 *>(b32 + p) = make_float2(bv[0], bv[1]);
            if constexpr (MODE == M_IR && KIND == GR_KIND_HAMILTONIAN) {
                *reinterpret_cast<float2 *>(a32 + p) = make_float2(av[0], av[1]);
                *reinterpret_cast<float2 *>(c32 + p) = make_float2(cv[0], cv[1]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                sr[j] += (MODE == M_RESTRICT) ? Lv[j] - (ff[j] - fs) : ff[j] - Lv[j];
                sp[j] += own_v[j];
            }
            if (z & 1) { // a z pair is complete: the x pair in this thread, the y pair across lanes
                T r2 = sr[0] + sr[1];
                T p2 = sp[0] + sp[1];
                r2 += __shfl_xor(r2, 32, 64);
                p2 += __shfl_xor(p2, 32, 64);
                if ((ty & 1) == 0) {
                    const int m = n >> 1;
                    const long q = ((long)(z >> 1) * m + ((y0 + ty) >> 1)) * m + (x0 >> 1) + tx;
                    if constexpr (MODE == M_RESTRICT) {
                        o1[q] = p2 / T(8); // R phi
                        o2[q] = p2 / T(8); // phi0
                        o3[q] = r2 / T(8); // R eps
                    } else {
                        o1[q] = r2 / T(8); // coarse b
                        o2[q] = T(0);      // coarse e
                    }
                }
                sr[0] = sr[1] = 0;
                sp[0] = sp[1] = 0;
            }
        }
        below = S.own;
        if (z + 2 < z0 + zc) load(S, z + 2);
        else if (z + 2 == z0 + zc) S.own = it2((long)wrapi(z + 2, n) * plane + own); // last plane's z + 1
    };
    for (int z = z0; z < z0 + zc; z += 2) {
        body(z, A, B);
        body(z + 1, B, A);
    }
    norm[0] = v0;
    norm[1] = v1;
}

} // namespace detail
} // namespace grmg
