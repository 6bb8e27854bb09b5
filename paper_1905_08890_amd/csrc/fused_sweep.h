// Fused red-black sweep of one tile x z-chunk (device function shared by the
// single-grid kernel and the batched kernel).  Included inside namespace
// grmg::(anonymous) after stencil_ops.h.
#pragma once

#include <type_traits>

#include "stencil_ops.h"

namespace grmg {
namespace detail {

// Fused red-black sweep, out of place (in -> out), both colours in one pass.
//
// A workgroup owns a TX x TY tile of (x, y) and marches a chunk of zc planes
// in z.  A 5-plane LDS ring holds `in` on the tile plus a 2-cell halo.  For
// each newly stored plane z it
//   1. updates the even (red) points of plane z-1 on the tile plus a 1-cell
//      halo, in place in LDS (red points only read odd neighbours, all old);
//   2. updates the odd (black) points of plane z-2 on the tile, whose
//      neighbours are the new red values of planes z-3..z-1, and writes both
//      colours of plane z-2 to `out` as 16-byte stores.
// Red values on the halo are recomputed from old data by every tile that needs
// them, so tiles never read each other's output: the result is exactly the
// red-then-black sweep, with phi read once and written once per sweep.
//
// Each thread owns one (even, odd) pair of x-points of a tile row: its red
// update is the red member of the pair, its black update the black member,
// and its source/coefficient values arrive as one 16-byte load per array that
// serves both (the black half waits one plane in registers), so every cache
// line of f and the coefficients is read once.  The 1-cell halo ring of red
// points (TX + TY + 2 per plane) is spread over the first threads with scalar
// loads.  All global reads of the next plane are issued into registers before
// the current plane's updates, so their latency overlaps the LDS work.  Five
// ring slots let the store of plane z+1 proceed without waiting for the black
// pass of z-2: two barriers per plane.
template <int KIND, typename T, int TX, int TY, int PF>
__device__ __forceinline__ void rb_fused_tile(const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ f,
                                              const T *__restrict__ c1, const T *__restrict__ c2, int n, int zc,
                                              T inv_h2, OpConst oc, const T Fb, const T fs, const int x0,
                                              const int y0, const int z0)
{
    constexpr int NT = (TX / 2) * TY;
    constexpr int W = TX + 4, H = TY + 4, PL = W * H;
    constexpr int NLOAD = (PL + NT - 1) / NT;
    constexpr int HALO = TX + TY + 2; // red points of the 1-cell halo ring, per plane
    static_assert(HALO <= NT, "halo ring larger than the workgroup");
    constexpr int NC = kNumCoef<KIND>();
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    __shared__ __align__(16) T ring[5][PL];

    const int tid = threadIdx.x;
    const int plane = n * n;
    const T rJ = poisson_inv_diag(inv_h2);

    // this thread's phi loads of a plane (tile + 2-halo)
    int goff[NLOAD];
    int lidx[NLOAD];
#pragma unroll
    for (int q = 0; q < NLOAD; ++q) {
        const int idx = tid + q * NT;
        lidx[q] = idx < PL ? idx : -1;
        const int ly = idx / W, lx = idx - ly * W;
        goff[q] = wrapi(y0 + ly - 2, n) * n + wrapi(x0 + lx - 2, n);
    }
    // this thread's pair: LDS row ly, even LDS column lxe; red member (x+y+z even) at lxe + ((ly + z) & 1)
    const int btx = tid % (TX / 2), bty = tid / (TX / 2);
    const int ly = 2 + bty, lxe = 2 + 2 * btx;
    const long pair_off = (long)(y0 + bty) * n + x0 + 2 * btx;
    // halo ring point h = tid (tid < HALO): LDS row/column for a plane z
    auto halo_pos = [&](int z, int &hy, int &hx) {
        const int h = tid;
        if (h < TX + 2) { // rows 1 and TY + 2, (TX + 2) / 2 red points each
            hy = h < (TX + 2) / 2 ? 1 : TY + 2;
            const int k = h < (TX + 2) / 2 ? h : h - (TX + 2) / 2;
            hx = 1 + ((hy + z + 1) & 1) + 2 * k;
        } else { // columns 1 and TX + 2 of rows 2..TY+1: one of the two is red
            hy = 2 + (h - (TX + 2));
            hx = ((1 + hy + z) & 1) == 0 ? 1 : TX + 2;
        }
    };
    auto halo_g = [&](int z, int hy, int hx) {
        return (long)wrapi(z, n) * plane + wrapi(y0 + hy - 2, n) * n + wrapi(x0 + hx - 2, n);
    };

    // Operands travel PF (1 to 4) planes ahead, in PF rotating register sets:
    // the iterate plane stored at iteration it was loaded at it - PF, and so
    // were the pair and halo values used by the red pass at it.
    struct Set {
        T pre[NLOAD];
        T2 f, c, a;
        T hf, hc, ha;
    };
    static_assert(PF >= 1 && PF <= 4, "prefetch depth 1 to 4");
    Set S[PF];
    // in == nullptr: the incoming iterate is identically zero (first sweep of a
    // correction cycle), so the plane loads are skipped
    const bool zero_in = in == nullptr;
    auto load_plane = [&](Set &S, int z) {
#pragma unroll
        for (int q = 0; q < NLOAD; ++q) S.pre[q] = T(0);
        if (!zero_in) {
            const T *src = in + (long)wrapi(z, n) * plane;
#pragma unroll
            for (int q = 0; q < NLOAD; ++q)
                if (lidx[q] >= 0) S.pre[q] = src[goff[q]];
        }
    };
    auto load_operands = [&](Set &S, int z) {
        const long gp = (long)wrapi(z, n) * plane + pair_off;
        S.f = *reinterpret_cast<const T2 *>(f + gp);
        if (NC >= 1) S.c = *reinterpret_cast<const T2 *>(c1 + gp);
        if (NC >= 2) S.a = *reinterpret_cast<const T2 *>(c2 + gp);
        if (tid < HALO) {
            int hy, hx;
            halo_pos(z, hy, hx);
            const long hg = halo_g(z, hy, hx);
            S.hf = f[hg];
            if (NC >= 1) S.hc = c1[hg];
            if (NC >= 2) S.ha = c2[hg];
        }
    };
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        S[q].f.x = S[q].f.y = S[q].c.x = S[q].c.y = S[q].a.x = S[q].a.y = S[q].hf = S[q].hc = S[q].ha = T(0);
        load_plane(S[q], z0 - 2 + q);
    }
    // the red pass at it (>= 2) works on plane z0 - 3 + it; below it = PF its
    // operands were not loaded inside the loop
#pragma unroll
    for (int q = 2; q < PF; ++q) load_operands(S[q], z0 - 3 + q);
    T fbk = 0, cbk = 0, abk = 0; // black half of the pair for the black pass of the next iteration

    int slot = 0; // slot of plane zz = z0 - 2 + it is it % 5
    auto body = [&](const int it, Set &R) {
        const int zz = z0 - 2 + it;
        T *cur = ring[slot];
#pragma unroll
        for (int q = 0; q < NLOAD; ++q)
            if (lidx[q] >= 0) cur[lidx[q]] = R.pre[q];
        __syncthreads();
        const bool ahead = it + PF < zc + 4;
        if (ahead) load_plane(R, zz + PF);
        const int s1 = slot == 0 ? 4 : slot - 1, s2 = s1 == 0 ? 4 : s1 - 1, s3 = s2 == 0 ? 4 : s2 - 1;
        if (it >= 2) { // red points of plane zr = zz - 1, tile + 1-cell halo
            const int zr = zz - 1;
            T *mid = ring[s1];
            const T *lo = ring[s2];
            const T *hi = ring[slot];
            const int o = (ly + zr) & 1; // red member of the pair
            {
                const int c = ly * W + lxe + o;
                const T ph = mid[c];
                const T nbs = mid[c - 1] + mid[c + 1] + mid[c - W] + mid[c + W] + lo[c] + hi[c];
                T J;
                const T L = op_point<KIND, T>(ph, nbs, inv_h2, o ? R.c.y : R.c.x, o ? R.a.y : R.a.x, oc, Fb, J);
                mid[c] = newton_update<KIND, T>(ph, L, (o ? R.f.y : R.f.x) - fs, J, rJ);
            }
            if (tid < HALO) {
                int hy, hx;
                halo_pos(zr, hy, hx);
                const int c = hy * W + hx;
                const T ph = mid[c];
                const T nbs = mid[c - 1] + mid[c + 1] + mid[c - W] + mid[c + W] + lo[c] + hi[c];
                T J;
                const T L = op_point<KIND, T>(ph, nbs, inv_h2, R.hc, R.ha, oc, Fb, J);
                mid[c] = newton_update<KIND, T>(ph, L, R.hf - fs, J, rJ);
            }
        }
        // plane zz - 1 had its red pass now; its black half is used at it + 1
        const int ob = (ly + zz) & 1;
        const T nfb = ob ? R.f.y : R.f.x, ncb = ob ? R.c.y : R.c.x, nab = ob ? R.a.y : R.a.x;
        if (ahead) load_operands(R, zz + PF - 1); // red pass of plane zz + PF - 1 at it + PF
        __syncthreads();
        if (it >= 4) { // black points of plane zb = zz - 2, tile only; write both colours
            const int zb = zz - 2;
            const T *mid = ring[s2];
            const T *lo = ring[s3];
            const T *hi = ring[s1];
            const int o = (ly + zb + 1) & 1; // black member of the pair
            const int c = ly * W + lxe + o;
            const T ph = mid[c];
            const T nbs = mid[c - 1] + mid[c + 1] + mid[c - W] + mid[c + W] + lo[c] + hi[c];
            T J;
            const T L = op_point<KIND, T>(ph, nbs, inv_h2, cbk, abk, oc, Fb, J);
            const T nb = newton_update<KIND, T>(ph, L, fbk - fs, J, rJ);
            const T red = mid[ly * W + lxe + (1 - o)];
            T2 v;
            v.x = o ? red : nb;
            v.y = o ? nb : red;
            *reinterpret_cast<T2 *>(out + (long)wrapi(zb, n) * plane + pair_off) = v;
        }
        fbk = nfb;
        cbk = ncb;
        abk = nab;
        slot = slot == 4 ? 0 : slot + 1;
    };
    for (int it = 0; it < zc + 4; it += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q)
            if (it + q < zc + 4) body(it + q, S[q]);
    }
}

} // namespace detail
} // namespace grmg
