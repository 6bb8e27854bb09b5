// Per-point device arithmetic of Dirichlet refinement patches (included
// inside namespace grmg::detail).
//
// A patch level of n^3 cells is stored padded, (n+2)^3 with x fastest; the
// cell across each boundary face holds that face's boundary value b, taken
// from the parent box at the face centre.  The 7-point stencil of a boundary
// cell uses 2b - phi_cell across the face (the linear extrapolation whose face
// average is b), the parent being a periodic box or (nested refinement) a
// patch, so the boundary sits on the same faces on every level and is
// second order.  Sources, coefficients and the restricted quantities stay
// dense n^3.  The paper takes the boundary values of refined levels from the
// coarser level (sec. 3) and regularises only the periodic equations
// (sec. 4.3.1, 4.3.2), so a patch solves the plain discrete equations.
#pragma once

#include "sources_ops.h"

namespace grmg {
namespace detail {

__device__ __forceinline__ long pidx(int i, int j, int k, int n)
{
    const long W = n + 2;
    return ((long)(k + 1) * W + (j + 1)) * W + (i + 1);
}

__device__ __forceinline__ int wrap_any(long i, int n)
{
    long r = i % n;
    return (int)(r < 0 ? r + n : r);
}

// Cell-centred trilinear interpolation of a periodic N^3 field of spacing H at
// the point (x, y, z): per axis g = x/H - 1/2, weights (1 - t, t) on cells
// floor(g) and floor(g) + 1 (wrapped), t = g - floor(g).
__device__ __forceinline__ double sample_periodic(const double *__restrict__ P, int N, double H, double x, double y,
                                                  double z)
{
    const double gx = x / H - 0.5, gy = y / H - 0.5, gz = z / H - 0.5;
    const double fx = floor(gx), fy = floor(gy), fz = floor(gz);
    const double t[3] = {gx - fx, gy - fy, gz - fz};
    const int i0[3] = {wrap_any((long)fx, N), wrap_any((long)fy, N), wrap_any((long)fz, N)};
    const int i1[3] = {i0[0] + 1 == N ? 0 : i0[0] + 1, i0[1] + 1 == N ? 0 : i0[1] + 1, i0[2] + 1 == N ? 0 : i0[2] + 1};
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz) {
        const double wz = cz ? t[2] : 1.0 - t[2];
        const int zz = cz ? i1[2] : i0[2];
        for (int cy = 0; cy < 2; ++cy) {
            const double wy = cy ? t[1] : 1.0 - t[1];
            const int yy = cy ? i1[1] : i0[1];
            for (int cx = 0; cx < 2; ++cx) {
                const double wx = cx ? t[0] : 1.0 - t[0];
                const int xx = cx ? i1[0] : i0[0];
                s += (wz * wy) * wx * P[lin(xx, yy, zz, N)];
            }
        }
    }
    return s;
}

// The same interpolation inside a parent patch (nested refinement): no wrap;
// the patch's placement was checked so that floor(g) and floor(g) + 1 are
// interior cells of the parent for every sample.  P is the parent's array,
// padded (n+2)^3 or dense n^3.
__device__ __forceinline__ double sample_inside(const double *__restrict__ P, int padded, int N, double H, double x,
                                                double y, double z)
{
    const double gx = x / H - 0.5, gy = y / H - 0.5, gz = z / H - 0.5;
    const double fx = floor(gx), fy = floor(gy), fz = floor(gz);
    const double t[3] = {gx - fx, gy - fy, gz - fz};
    const int i0[3] = {(int)fx, (int)fy, (int)fz};
    double s = 0.0;
    for (int cz = 0; cz < 2; ++cz) {
        const double wz = cz ? t[2] : 1.0 - t[2];
        const int zz = i0[2] + cz;
        for (int cy = 0; cy < 2; ++cy) {
            const double wy = cy ? t[1] : 1.0 - t[1];
            const int yy = i0[1] + cy;
            for (int cx = 0; cx < 2; ++cx) {
                const double wx = cx ? t[0] : 1.0 - t[0];
                const int xx = i0[0] + cx;
                s += (wz * wy) * wx * P[padded ? pidx(xx, yy, zz, N) : lin(xx, yy, zz, N)];
            }
        }
    }
    return s;
}

// A parent's field at a point of its frame: periodic box or patch
__device__ __forceinline__ double sample_parent_at(const double *__restrict__ P, int parent_is_patch, int padded,
                                                   int N, double H, double x, double y, double z)
{
    return parent_is_patch ? sample_inside(P, padded, N, H, x, y, z) : sample_periodic(P, N, H, x, y, z);
}

// A patch field for the source builders: the patch's own value inside, the
// parent's field at the cell centre outside (one cell beyond the faces, edges
// and corners included).
struct PatchField {
    const double *p; // patch array: padded (n+2)^3 or dense n^3
    int padded;
    int n;
    double h, ox, oy, oz; // level-0 spacing and lower corner in the parent's frame
    const double *parent;
    int N;
    double H;
    int ppatch, ppadded; // parent is a patch; its array is padded
    __device__ __forceinline__ double operator()(int i, int j, int k) const
    {
        if ((unsigned)i < (unsigned)n && (unsigned)j < (unsigned)n && (unsigned)k < (unsigned)n)
            return p[padded ? pidx(i, j, k, n) : lin(i, j, k, n)];
        return sample_parent_at(parent, ppatch, ppadded, N, H, ox + (i + 0.5) * h, oy + (j + 0.5) * h,
                                oz + (k + 0.5) * h);
    }
};

// L(phi) at interior cell (i,j,k) of a padded patch level and dL/dphi there;
// no regularisation terms (Fbar = 0, no source shift).
template <int KIND>
__device__ __forceinline__ double patch_op(const double *__restrict__ phi, int i, int j, int k, int n, double inv_h2,
                                           double c1, OpConst oc, double &J)
{
    const long W = n + 2, W2 = W * W, p = pidx(i, j, k, n);
    const double ph = phi[p];
    double nbs = phi[p - 1] + phi[p + 1] + phi[p - W] + phi[p + W] + phi[p - W2] + phi[p + W2];
    int nf = 0;
    // across a boundary face use 2b - phi_cell: b is stored there, add b - phi_cell
    if (i == 0) { nbs += phi[p - 1] - ph; ++nf; }
    if (i == n - 1) { nbs += phi[p + 1] - ph; ++nf; }
    if (j == 0) { nbs += phi[p - W] - ph; ++nf; }
    if (j == n - 1) { nbs += phi[p + W] - ph; ++nf; }
    if (k == 0) { nbs += phi[p - W2] - ph; ++nf; }
    if (k == n - 1) { nbs += phi[p + W2] - ph; ++nf; }
    const double L = op_point<KIND, double>(ph, nbs, inv_h2, c1, 0.0, oc, 0.0, J);
    // the extrapolated neighbours depend on phi_cell too
    if (nf) J -= (double)nf * inv_h2 * (KIND == GR_KIND_HAMILTONIAN ? 1.0 - oc.kappa * ph : 1.0);
    return L;
}

// The prolonged coarse correction continues oddly across every face: its
// value at coarse index I outside [0, m) is minus (per axis) that of the
// adjacent inside cell.
__device__ __forceinline__ int reflect_in(int I, int m, double &sign)
{
    if (I < 0) {
        sign = -sign;
        return 0;
    }
    if (I >= m) {
        sign = -sign;
        return m - 1;
    }
    return I;
}

} // namespace detail
} // namespace grmg
