// Multigrid stencil kernels for gfx950: red-black pointwise-Newton
// Gauss-Seidel smoother, fused residual + restriction, FAS coarse source,
// trilinear prolongation + correction, and deterministic reductions.
//
// Equations (paper sec. 4.3): 7-point Laplacian Lap_h; operators
//   Poisson     L = Lap phi
//   Hamiltonian L = chi Lap Psi + A (chi^6 - 1) - AA chi^-6 / 4 + Fbar chi,
//               chi = 1 - kappa Psi, A = 3/2 a Om, Fbar = <F> (finest level only)
//   CMC         L = Lap xi - m2 xi, source shifted by fshift = <f> + <m2 xi>
// The Newton step per point is phi <- phi - (L - f)/(dL/dphi) with the
// neighbours held fixed (exact Gauss-Seidel for the linear kinds).
//
// The same kernels, instantiated in FP32 with the linearised operators
// J e = a Lap e + c e (kinds K_LIN_*), run the inner correction cycles of
// mixed-precision iterative refinement: Poisson a = 1, c = 0; Hamiltonian
// a = chi, c = dL/dPsi - chi dLap/dPsi; CMC a = 1, c = -m2.
#include <cstdlib>
#include <type_traits>

#include "stencil_ops.h"
#include "fused_sweep.h"
#include "coarse_cycle.h"
#include "march.h"

namespace grmg {

namespace {

constexpr int TPB = 256;
using namespace detail;

// 3-D launch geometry for an nx x ny x nz domain: x across the threads of a
// block (up to 64), y across threadIdx.y/blockIdx.y, z = blockIdx.z.
struct Geo {
    dim3 grid, block;
};
inline Geo geo3(int nx, int ny, int nz)
{
    const int bx = nx < 64 ? nx : 64;
    int by = TPB / bx;
    if (by > ny) by = ny;
    Geo g;
    g.block = dim3(bx, by, 1);
    g.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nz);
    return g;
}

#define GEO_XYZ(nx, ny)                                                                               \
    const int x = blockIdx.x * blockDim.x + threadIdx.x;                                              \
    const int y = blockIdx.y * blockDim.y + threadIdx.y;                                              \
    const int z = blockIdx.z;                                                                         \
    if (x >= (nx) || y >= (ny)) return;

// ----------------------------------------------------------------- smoother

// One colour of a red-black sweep; one thread per point of that colour.
// Colour c holds (i+j+k) % 2 == c; consecutive threads take consecutive
// same-colour points of one x-row.
template <int KIND, typename T>
__global__ void __launch_bounds__(TPB) k_rb_colour(T *__restrict__ phi, const T *__restrict__ f,
                                                   const T *__restrict__ c1, const T *__restrict__ c2, int n,
                                                   T inv_h2, int colour, OpConst oc, const double *__restrict__ fbar,
                                                   const double *__restrict__ fshift)
{
    GEO_XYZ(n >> 1, n)
    const int i = 2 * x + ((y + z + colour) & 1);
    const long p = lin(i, y, z, n);
    const T ph = phi[p];
    T J;
    const T L = op_point<KIND, T>(ph, nb_sum(phi, i, y, z, n), inv_h2, load_c1<KIND>(c1, p), load_c2<KIND>(c2, p),
                                  oc, T(*fbar), J);
    phi[p] = newton_update<KIND, T>(ph, L, f[p] - T(*fshift), J, poisson_inv_diag(inv_h2));
}

// One workgroup per tile x z-chunk of the single grid (see rb_fused_tile).
template <int KIND, typename T, int TX, int TY, int PF>
__global__ void __launch_bounds__((TX / 2) * TY) k_rb_fused(
    const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ f, const T *__restrict__ c1,
    const T *__restrict__ c2, int n, int zc, T inv_h2, OpConst oc, const double *__restrict__ fbar,
    const double *__restrict__ fshift, int tiles_y, int xcd_remap)
{
    int b = blockIdx.x;
    const int G = gridDim.x;
    const int nz = n / zc;
    int zchunk, tx, ty;
    if (xcd_remap == 2 && (G & 7) == 0) {
        // Workgroups are dispatched to the 8 XCDs in turn: give XCD b % 8 a
        // contiguous run of G / 8 tiles of one z-chunk, x fastest, so the
        // halos the tiles exchange are fetched into that XCD's own L2 once.
        const int w = (b & 7) * (G >> 3) + (b >> 3);
        const int per_plane = G / nz, tiles_x = per_plane / tiles_y, t = w % per_plane;
        zchunk = w / per_plane;
        tx = t % tiles_x;
        ty = t / tiles_x;
    } else {
        if (xcd_remap == 1 && (G & 7) == 0) b = (b & 7) * (G >> 3) + (b >> 3); // one XCD gets a contiguous range
        zchunk = b % nz;
        const int t2 = b / nz;
        tx = t2 / tiles_y;
        ty = t2 % tiles_y;
    }
    rb_fused_tile<KIND, T, TX, TY, PF>(in, out, f, c1, c2, n, zc, inv_h2, oc, T(*fbar), T(*fshift), tx * TX, ty * TY,
                                       zchunk * zc);
}

// ------------------------------------------------- residual and restriction

// One thread per coarse cell: residual at the 8 children, their mean (R eps),
// and the mean of the children of phi (R phi, also saved as phi0).
template <int KIND>
__global__ void __launch_bounds__(TPB) k_residual_restrict(
    const double *__restrict__ phi, const double *__restrict__ f, const double *__restrict__ coef, int n,
    double inv_h2, OpConst oc, const double *__restrict__ fbar, const double *__restrict__ fshift,
    double *__restrict__ phi_c, double *__restrict__ phi0_c, double *__restrict__ rr_c)
{
    const int m = n >> 1;
    GEO_XYZ(m, m)
    const double Fb = *fbar, fs = *fshift;
    double sr = 0.0, sp = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * x + (c & 1), j = 2 * y + ((c >> 1) & 1), k = 2 * z + (c >> 2);
        const long p = lin(i, j, k, n);
        const double ph = phi[p];
        double Jd;
        const double L = op_point<KIND, double>(ph, nb_sum(phi, i, j, k, n), inv_h2, load_c1<KIND>(coef, p), 0.0,
                                                oc, Fb, Jd);
        sr += L - (f[p] - fs);
        sp += ph;
    }
    const long q = lin(x, y, z, m);
    const double rp = sp / 8.0;
    phi_c[q] = rp;
    phi0_c[q] = rp;
    rr_c[q] = sr / 8.0;
}

// FAS coarse source f^H = L^H(R phi) - R eps (coarse operator: unregularised).
template <int KIND>
__global__ void __launch_bounds__(TPB) k_coarse_rhs(const double *__restrict__ phi_c,
                                                    const double *__restrict__ coef_c,
                                                    const double *__restrict__ rr_c, int m, double inv_H2,
                                                    OpConst oc, double *__restrict__ f_c)
{
    GEO_XYZ(m, m)
    const long q = lin(x, y, z, m);
    double Jd;
    const double L = op_point<KIND, double>(phi_c[q], nb_sum(phi_c, x, y, z, m), inv_H2, load_c1<KIND>(coef_c, q),
                                            0.0, oc, 0.0, Jd);
    f_c[q] = L - rr_c[q];
}

// Residual of one level into r (used by the step-by-step entry point).
template <int KIND>
__global__ void __launch_bounds__(TPB) k_residual(const double *__restrict__ phi, const double *__restrict__ f,
                                                  const double *__restrict__ coef, int n, double inv_h2,
                                                  OpConst oc, const double *__restrict__ fbar,
                                                  const double *__restrict__ fshift, double *__restrict__ r)
{
    GEO_XYZ(n, n)
    const long p = lin(x, y, z, n);
    double Jd;
    const double L = op_point<KIND, double>(phi[p], nb_sum(phi, x, y, z, n), inv_h2, load_c1<KIND>(coef, p), 0.0,
                                            oc, *fbar, Jd);
    r[p] = L - (f[p] - *fshift);
}

// Restriction of an arbitrary array: mean of the 8 children.
template <typename T>
__global__ void __launch_bounds__(TPB) k_restrict(const T *__restrict__ fine, int n, T *__restrict__ coarse)
{
    const int m = n >> 1;
    GEO_XYZ(m, m)
    T s = 0;
    for (int c = 0; c < 8; ++c) s += fine[lin(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2), n)];
    coarse[lin(x, y, z, m)] = s / T(8);
}

// Linear correction scheme: coarse source b^H = R(b - J e) and coarse e^H = 0.
template <int KIND, typename T>
__global__ void __launch_bounds__(TPB) k_lin_residual_restrict(const T *__restrict__ e, const T *__restrict__ b,
                                                               const T *__restrict__ c1, const T *__restrict__ c2,
                                                               int n, T inv_h2, OpConst oc, T *__restrict__ b_c,
                                                               T *__restrict__ e_c)
{
    const int m = n >> 1;
    GEO_XYZ(m, m)
    T sr = 0;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * x + (c & 1), j = 2 * y + ((c >> 1) & 1), k = 2 * z + (c >> 2);
        const long p = lin(i, j, k, n);
        T Jd;
        const T L = op_point<KIND, T>(e[p], nb_sum(e, i, j, k, n), inv_h2, load_c1<KIND>(c1, p), load_c2<KIND>(c2, p),
                                      oc, T(0), Jd);
        sr += b[p] - L;
    }
    const long q = lin(x, y, z, m);
    b_c[q] = sr / T(8);
    e_c[q] = T(0);
}

// Cell-centred trilinear prolongation of the coarse correction, added in
// place: e = phi_c - phi0_c (FAS) or e = phi_c (correction scheme).  Fine cell
// 2I takes 3/4 of coarse cell I and 1/4 of I-1, fine cell 2I+1 takes 3/4 of I
// and 1/4 of I+1 (per axis, periodic).  One thread per coarse (x, y) column
// marches a chunk of zc coarse planes: the 3 x 3 neighbourhood of the three
// coarse planes around the current one stays in registers (one new plane of 9
// values per step), and the thread writes the 8 children of its coarse cell
// (x-pairs as one 16-byte read-modify-write).
template <typename T, bool FAS>
__global__ void __launch_bounds__(TPB) k_prolong_correct(T *__restrict__ phi_f, int n, int zc,
                                                         const T *__restrict__ phi_c, const T *__restrict__ phi0_c)
{
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
    const int m = n >> 1;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x >= m || y >= m) return;
    const int z0 = blockIdx.z * zc;
    const int xm = wrapi(x - 1, m), xp = wrapi(x + 1, m);
    const int ym = wrapi(y - 1, m), yp = wrapi(y + 1, m);
    const int xs[3] = {xm, x, xp}, ys[3] = {ym, y, yp};
    T e[3][3][3]; // e[dz+1][dy+1][dx+1]
    auto load_plane = [&](T(&pl)[3][3], int zz) {
        const long zo = (long)wrapi(zz, m) * m;
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
                const long q = (zo + ys[dy]) * m + xs[dx];
                pl[dy][dx] = FAS ? phi_c[q] - phi0_c[q] : phi_c[q];
            }
    };
    load_plane(e[0], z0 - 1);
    load_plane(e[1], z0);
    for (int z = z0; z < z0 + zc; ++z) {
        // the four fine x-pairs of this coarse cell are read before the next
        // coarse plane, so all thirteen (FAS: twenty-two) loads are in flight at once
        T2 old[2][2];
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                old[cz][cy] = *reinterpret_cast<const T2 *>(phi_f + lin(2 * x, 2 * y + cy, 2 * z + cz, n));
        load_plane(e[2], z + 1);
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy) {
                T v[2];
                for (int cx = 0; cx < 2; ++cx) {
                    const int sx = cx ? 1 : -1, sy = cy ? 1 : -1, sz = cz ? 1 : -1;
                    T a = 0;
                    for (int c = 0; c < 8; ++c) {
                        const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                        const T w = (ox ? T(0.25) : T(0.75)) * (oy ? T(0.25) : T(0.75)) * (oz ? T(0.25) : T(0.75));
                        a += w * e[1 + oz * sz][1 + oy * sy][1 + ox * sx];
                    }
                    v[cx] = a;
                }
                T2 r = old[cz][cy];
                r.x += v[0];
                r.y += v[1];
                *reinterpret_cast<T2 *>(phi_f + lin(2 * x, 2 * y + cy, 2 * z + cz, n)) = r;
            }
        for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
                e[0][dy][dx] = e[1][dy][dx];
                e[1][dy][dx] = e[2][dy][dx];
            }
    }
}

// grid of k_prolong_correct for fine side n: coarse columns in 64 x 4 blocks,
// z-chunks of the largest of 8, 4, 2, 1 planes that divides the coarse side
// and still leaves at least 128 Ki threads (small levels: parallelism first)
struct ProlongGeo {
    dim3 grid, block;
    int zc;
};
inline ProlongGeo prolong_geo(int n)
{
    const int m = n / 2;
    const int bx = m < 64 ? m : 64;
    int by = 256 / bx;
    if (by > m) by = m;
    static const int zmax = [] {
        const char *e = std::getenv("GRMG_PROLONG_ZC");
        const int v = e ? std::atoi(e) : 8;
        return v >= 8 ? 8 : (v >= 4 ? 4 : (v >= 2 ? 2 : 1));
    }();
    int zc = zmax;
    while (zc > 1 && (m % zc != 0 || (long)m * m * (m / zc) < 131072L)) zc /= 2;
    ProlongGeo g;
    g.block = dim3(bx, by, 1);
    g.grid = dim3((m + bx - 1) / bx, (m + by - 1) / by, m / zc);
    g.zc = zc;
    return g;
}

// ----------------------------------------------------------------- reductions

// Block-level sum of NC values per thread, fixed order: wavefront shuffles
// (64 lanes) then the waves of the block in order.
template <int NC>
__device__ __forceinline__ void block_sum_store(double (&v)[NC], double *__restrict__ partials)
{
    __shared__ double sh[NC][TPB / 64];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = v[c];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[c][wave] = x;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int w = 0; w < TPB / 64; ++w) s += sh[c][w];
            partials[c * kReduceBlocks + blockIdx.x] = s;
        }
    }
}

// Plain sums over n^3 arrays.  Each thread adds consecutive pairs (one 16-byte
// load per array) in a grid-stride loop over the pairs when the arrays allow it
// (N even, 16-byte aligned), else single elements; the number of workgroups
// (at most kReduceBlocks) depends only on N, so the order of the additions,
// and the result, is fixed for a given size.  Block 0 zeroes the partial-sum
// slots of the workgroups not launched.
inline unsigned reduce_blocks(long N)
{
    long b = (N + 8L * TPB - 1) / (8L * TPB);
    return (unsigned)(b < 1 ? 1 : (b > kReduceBlocks ? kReduceBlocks : b));
}

template <int NC>
__device__ __forceinline__ void zero_unused_partials(double *__restrict__ partials)
{
    if (blockIdx.x == 0)
        for (int b = gridDim.x + threadIdx.x; b < kReduceBlocks; b += blockDim.x * blockDim.y)
#pragma unroll
            for (int c = 0; c < NC; ++c) partials[c * kReduceBlocks + b] = 0.0;
}

// sum of x (pair: 1) or of x - y
template <typename F>
__device__ __forceinline__ double sum_pairs(long N, bool pair, F term)
{
    double v = 0.0;
    const long stride = (long)gridDim.x * TPB;
    if (pair) {
        for (long q = (long)blockIdx.x * TPB + threadIdx.x; q < N / 2; q += stride) v = term(2 * q, v, true);
    } else {
        for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < N; p += stride) v = term(p, v, false);
    }
    return v;
}

__global__ void __launch_bounds__(TPB) k_sum(const double *__restrict__ x, const double *__restrict__ y, long N,
                                             bool pair, double *__restrict__ partials)
{
    double v[1];
    v[0] = sum_pairs(N, pair, [&](long p, double acc, bool two) {
        if (two) {
            const double2 a = *reinterpret_cast<const double2 *>(x + p);
            if (y) {
                const double2 b = *reinterpret_cast<const double2 *>(y + p);
                acc += a.x - b.x;
                acc += a.y - b.y;
            } else {
                acc += a.x;
                acc += a.y;
            }
            return acc;
        }
        return acc + (y ? (x[p] - y[p]) : x[p]);
    });
    block_sum_store<1>(v, partials);
    zero_unused_partials<1>(partials);
}

__global__ void __launch_bounds__(TPB) k_sum_prod(const double *__restrict__ x, const double *__restrict__ y,
                                                  long N, bool pair, double *__restrict__ partials)
{
    double v[1];
    v[0] = sum_pairs(N, pair, [&](long p, double acc, bool two) {
        if (two) {
            const double2 a = *reinterpret_cast<const double2 *>(x + p);
            const double2 b = *reinterpret_cast<const double2 *>(y + p);
            acc += a.x * b.x;
            acc += a.y * b.y;
            return acc;
        }
        return acc + x[p] * y[p];
    });
    block_sum_store<1>(v, partials);
    zero_unused_partials<1>(partials);
}

// F = (f - A(chi^6 - 1))/chi + AA chi^-7/4 (Hamiltonian regulariser) at one point
__device__ __forceinline__ double ham_F(double psi, double f, double AA, OpConst oc)
{
    const double chi = 1.0 - oc.kappa * psi;
    const double chi2 = chi * chi;
    const double chi6 = chi2 * chi2 * chi2;
    const double chim7 = 1.0 / (chi6 * chi);
    return (f - oc.A * (chi6 - 1.0)) / chi + 0.25 * AA * chim7;
}

// Sum of F over the grid.
__global__ void __launch_bounds__(TPB) k_sum_ham_F(const double *__restrict__ psi, const double *__restrict__ f,
                                                   const double *__restrict__ coef, long N, OpConst oc, bool pair,
                                                   double *__restrict__ partials)
{
    double v[1];
    v[0] = sum_pairs(N, pair, [&](long p, double acc, bool two) {
        if (two) {
            const double2 a = *reinterpret_cast<const double2 *>(psi + p);
            const double2 b = *reinterpret_cast<const double2 *>(f + p);
            const double2 c = *reinterpret_cast<const double2 *>(coef + p);
            acc += ham_F(a.x, b.x, c.x, oc);
            acc += ham_F(a.y, b.y, c.y, oc);
            return acc;
        }
        return acc + ham_F(psi[p], f[p], coef[p], oc);
    });
    block_sum_store<1>(v, partials);
    zero_unused_partials<1>(partials);
}

// The FP64 update of a refinement step, phi <- phi + e - <e>, fused with the
// pass that follows it: the sum of F (Hamiltonian, coef = AA) or of coef * phi
// (CMC, coef = m2) over the updated field.  Same thread mapping and order of
// additions as k_sum_ham_F / k_sum_prod, and the update of EwIrUpdate, so the
// fused pass gives the two separate passes' field and partial sums bit for bit.
template <bool HAM>
__global__ void __launch_bounds__(TPB) k_ir_update_sum(double *__restrict__ phi, const float *__restrict__ e,
                                                       const double *__restrict__ mean, const double *__restrict__ f,
                                                       const double *__restrict__ coef, long N, OpConst oc, bool pair,
                                                       double *__restrict__ partials)
{
    const double m = *mean;
    double v[1];
    v[0] = sum_pairs(N, pair, [&](long p, double acc, bool two) {
        if (two) {
            double2 a = *reinterpret_cast<const double2 *>(phi + p);
            const float2 u = *reinterpret_cast<const float2 *>(e + p);
            a.x += (double)u.x - m;
            a.y += (double)u.y - m;
            *reinterpret_cast<double2 *>(phi + p) = a;
            const double2 c = *reinterpret_cast<const double2 *>(coef + p);
            if constexpr (HAM) {
                const double2 b = *reinterpret_cast<const double2 *>(f + p);
                acc += ham_F(a.x, b.x, c.x, oc);
                acc += ham_F(a.y, b.y, c.y, oc);
            } else {
                acc += c.x * a.x;
                acc += c.y * a.y;
            }
            return acc;
        }
        double a = phi[p];
        a += (double)e[p] - m;
        phi[p] = a;
        return HAM ? acc + ham_F(a, f[p], coef[p], oc) : acc + coef[p] * a;
    });
    block_sum_store<1>(v, partials);
    zero_unused_partials<1>(partials);
}

// Both linearisation arrays (a and c of the FP32 Hamiltonian correction)
// restricted one level in one launch (the per-element arithmetic of k_restrict).
__global__ void __launch_bounds__(TPB) k_restrict2(const float *__restrict__ fa, const float *__restrict__ fc, int n,
                                                   float *__restrict__ ca, float *__restrict__ cc)
{
    const int m = n >> 1;
    GEO_XYZ(m, m)
    float sa = 0, sc = 0;
    for (int c = 0; c < 8; ++c) {
        const long q = lin(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2), n);
        sa += fa[q];
        sc += fc[q];
    }
    ca[lin(x, y, z, m)] = sa / 8.f;
    cc[lin(x, y, z, m)] = sc / 8.f;
}

// The same for the levels from side n down to side 2, in one workgroup (levels
// of at most 32^3: one launch instead of one per level and array).
__global__ void __launch_bounds__(kCoarseThreads) k_restrict2_chain(RestrictChain R)
{
    for (int l = 0; l < R.nl; ++l) {
        const int n = R.n[l], m = n >> 1, M = m * m * m;
        for (int q = threadIdx.x; q < M; q += kCoarseThreads) {
            const int x = q % m, y = (q / m) % m, z = q / (m * m);
            float sa = 0, sc = 0;
            for (int c = 0; c < 8; ++c) {
                const long p = lin(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + (c >> 2), n);
                sa += R.a[l][p];
                sc += R.c[l][p];
            }
            R.a[l + 1][q] = sa / 8.f;
            R.c[l + 1][q] = sc / 8.f;
        }
        __syncthreads();
    }
}

// Sums of eps^2 and (f - fshift)^2 on one level.  Blocks of 64 x 4 threads
// walk x-rows (row r = (y, z)) in a grid-stride loop over the n^2 rows.
template <int KIND>
__global__ void __launch_bounds__(TPB) k_res_norms(const double *__restrict__ phi, const double *__restrict__ f,
                                                   const double *__restrict__ coef, int n, double inv_h2,
                                                   OpConst oc, const double *__restrict__ fbar,
                                                   const double *__restrict__ fshift,
                                                   double *__restrict__ partials)
{
    const double Fb = *fbar, fs = *fshift;
    double v[2] = {0.0, 0.0};
    const int rows = n * n;
    for (int r = blockIdx.x * 4 + threadIdx.y; r < rows; r += gridDim.x * 4) {
        const int y = r % n, z = r / n;
        for (int x = threadIdx.x; x < n; x += 64) {
            const long p = lin(x, y, z, n);
            double Jd;
            const double L = op_point<KIND, double>(phi[p], nb_sum(phi, x, y, z, n), inv_h2, load_c1<KIND>(coef, p),
                                                    0.0, oc, Fb, Jd);
            const double fe = f[p] - fs;
            const double e = L - fe;
            v[0] += e * e;
            v[1] += fe * fe;
        }
    }
    block_sum_store<2>(v, partials);
    zero_unused_partials<2>(partials);
}

// out[c] = (add ? add[c] : 0) + scale * sum of partials of component c, in a
// fixed order (one block; thread t sums blocks t, t+256, ... then a tree).
// Fixed-order sum of the block partials of up to two quantities: every thread
// adds its 16 strided slots in slot order, then a tree over the threads (pairs
// t, t + w for w = 128, 64, ..., 1).  All loads are issued before the first
// add (the partials were just written by other XCDs and come from memory, so a
// load-add chain would pay that latency 16 times); the last six tree levels run
// in the first wavefront by lane shuffles, which pair the same values.
constexpr int kFinalizeSlots = kReduceBlocks / TPB;

__global__ void __launch_bounds__(TPB) k_finalize(const double *__restrict__ partials, int ncomp, double scale,
                                                  const double *__restrict__ add, double *__restrict__ out,
                                                  double *__restrict__ host_out)
{
    __shared__ double sh[2][TPB];
    double v[2][kFinalizeSlots];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < kFinalizeSlots; ++j)
            v[c][j] = c < ncomp ? partials[c * kReduceBlocks + j * TPB + threadIdx.x] : 0.0;
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < kFinalizeSlots; ++j) s += v[c][j];
        sh[c][t] = s;
    }
    __syncthreads();
    for (int w = TPB / 2; w >= 64; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    if (t < 64) {
        double s0 = sh[0][t], s1 = sh[1][t];
        for (int w = 32; w > 0; w >>= 1) {
            s0 += __shfl_down(s0, w, 64);
            s1 += __shfl_down(s1, w, 64);
        }
        if (t == 0) {
            const double r0 = (add ? add[0] : 0.0) + scale * s0, r1 = (add ? add[1] : 0.0) + scale * s1;
            out[0] = r0;
            if (ncomp > 1) out[1] = r1;
            if (host_out) { // straight to the host's page-locked slots (no read-back copy)
                host_out[0] = r0;
                if (ncomp > 1) host_out[1] = r1;
                __threadfence_system();
            }
        }
    }
}

// ------------------------------------------ plane-marching residual kernels
// (march_tile: one workgroup per 32 x 8 tile and z-chunk)

template <int MODE, int KIND, typename T>
__global__ void __launch_bounds__(MNT) k_march(const T *__restrict__ phi, const T *__restrict__ f,
                                               const T *__restrict__ c1, const T *__restrict__ c2, int n, int zc,
                                               T inv_h2, OpConst oc, const double *__restrict__ fbar,
                                               const double *__restrict__ fshift, double *__restrict__ partials,
                                               T *__restrict__ o1, T *__restrict__ o2, T *__restrict__ o3,
                                               float *__restrict__ b32, float *__restrict__ a32,
                                               float *__restrict__ c32, const float *__restrict__ e32)
{
    const int tiles_y = n / MTY;
    const int nzc = n / zc;
    const int tile = blockIdx.x / nzc, zchunk = blockIdx.x % nzc;
    const T Fb = (MODE == M_RESTRICT_LIN) ? T(0) : T(*fbar);
    const T fs = (MODE == M_RESTRICT_LIN) ? T(0) : T(*fshift);
    double v[2] = {0.0, 0.0};
    march_tile<MODE, KIND, T>(phi, f, c1, c2, n, zc, inv_h2, oc, Fb, fs, (tile / tiles_y) * MTX,
                              (tile % tiles_y) * MTY, zchunk * zc, o1, o2, o3, b32, a32, c32, v, e32);
    if constexpr (MODE == M_NORMS || MODE == M_IR || MODE == M_IRU) {
        block_sum_store<2>(v, partials);
        if (blockIdx.x == 0) // unused partial slots of a smaller grid
            for (int b2 = gridDim.x + threadIdx.x; b2 < kReduceBlocks; b2 += MNT) {
                partials[b2] = 0.0;
                partials[kReduceBlocks + b2] = 0.0;
            }
    }
}

// The same passes on 64 x 8 tiles with x-pairs per thread (march_tile2): levels
// with n a multiple of 64.
template <int MODE, int KIND, typename T>
__global__ void __launch_bounds__(M2NT) k_march2(const T *__restrict__ phi, const T *__restrict__ f,
                                                 const T *__restrict__ c1, const T *__restrict__ c2, int n, int zc_arg,
                                                 T inv_h2, OpConst oc, const double *__restrict__ fbar,
                                                 const double *__restrict__ fshift, double *__restrict__ partials,
                                                 T *__restrict__ o1, T *__restrict__ o2, T *__restrict__ o3,
                                                 float *__restrict__ b32, float *__restrict__ a32,
                                                 float *__restrict__ c32, const float *__restrict__ e32)
{
    const int tiles_y = n / M2TY;
    const int zc = zc_arg & 0xffff;
    const int nzc = n / zc;
    int tile, zchunk;
    if (zc_arg >> 16) { // z-chunk major in contiguous runs per XCD: tile neighbours in x, y and z share an L2
        const int G = gridDim.x, ntiles = G / nzc;
        const int v = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
        zchunk = v / ntiles;
        tile = v - zchunk * ntiles;
    } else {
        tile = blockIdx.x / nzc;
        zchunk = blockIdx.x % nzc;
    }
    const T Fb = (MODE == M_RESTRICT_LIN) ? T(0) : T(*fbar);
    const T fs = (MODE == M_RESTRICT_LIN) ? T(0) : T(*fshift);
    double v[2] = {0.0, 0.0};
    march_tile2<MODE, KIND, T>(phi, f, c1, c2, n, zc, inv_h2, oc, Fb, fs, (tile / tiles_y) * M2TX,
                               (tile % tiles_y) * M2TY, zchunk * zc, o1, o2, o3, b32, a32, c32, v, e32);
    if constexpr (MODE == M_NORMS || MODE == M_IR || MODE == M_IRU) {
        block_sum_store<2>(v, partials);
        zero_unused_partials<2>(partials);
    }
}

// ------------------------------------------------- coarse levels, one block

constexpr int CTPB = kCoarseThreads;

template <int KIND, typename T>
__global__ void __launch_bounds__(CTPB) k_coarse_vcycle(CoarseLevelsT<T> C, int nu1, int nu2, OpConst oc,
                                                        const double *__restrict__ fbar0,
                                                        const double *__restrict__ fshift0)
{
    coarse_vcycle_body<KIND, T>(C, nu1, nu2, oc, T(*fbar0), T(*fshift0));
}

template <int KIND, typename TG, typename T>
__global__ void __launch_bounds__(CTPB) k_coarse_vcycle_lds(CoarseLevelsT<TG> G, int nu1, int nu2, OpConst oc,
                                                            const double *__restrict__ fbar0,
                                                            const double *__restrict__ fshift0)
{
    coarse_cycle_lds<KIND, TG, T>(G, nu1, nu2, oc, fbar0, fshift0);
}

// ------------------------------------------------ mixed-precision outer steps

// FP64 fine residual r = L(phi) - (f - fshift) of a FAS kind; writes the
// FP32 correction source b = -r and, for the Hamiltonian, the frozen
// linearisation a = chi and c = dL/dPsi + 6 chi/h^2; accumulates sums of
// r^2 and (f - fshift)^2 for the stopping test.
template <int KIND>
__global__ void __launch_bounds__(TPB) k_ir_residual(const double *__restrict__ phi, const double *__restrict__ f,
                                                     const double *__restrict__ coef, int n, double inv_h2,
                                                     OpConst oc, const double *__restrict__ fbar,
                                                     const double *__restrict__ fshift, float *__restrict__ b32,
                                                     float *__restrict__ a32, float *__restrict__ c32,
                                                     double *__restrict__ partials)
{
    const double Fb = *fbar, fs = *fshift;
    double v[2] = {0.0, 0.0};
    const int rows = n * n;
    for (int r = blockIdx.x * 4 + threadIdx.y; r < rows; r += gridDim.x * 4) {
        const int y = r % n, z = r / n;
        for (int x = threadIdx.x; x < n; x += 64) {
            const long p = lin(x, y, z, n);
            const double ph = phi[p];
            double J;
            const double L = op_point<KIND, double>(ph, nb_sum(phi, x, y, z, n), inv_h2, load_c1<KIND>(coef, p), 0.0,
                                                    oc, Fb, J);
            const double fe = f[p] - fs;
            const double e = L - fe;
            v[0] += e * e;
            v[1] += fe * fe;
            b32[p] = (float)(-e);
            if constexpr (KIND == GR_KIND_HAMILTONIAN) {
                const double chi = 1.0 - oc.kappa * ph;
                a32[p] = (float)chi;
                c32[p] = (float)(J + 6.0 * chi * inv_h2);
            }
        }
    }
    block_sum_store<2>(v, partials);
    zero_unused_partials<2>(partials);
}

// c = -m2 in FP32 (linearised CMC coefficient; fixed for the whole solve)
__global__ void k_neg_to_f32(float *__restrict__ d, const double *__restrict__ s, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = (float)(-s[p]);
}

__global__ void __launch_bounds__(TPB) k_sum_f32(const float *__restrict__ x, long N, bool pair,
                                                 double *__restrict__ partials)
{
    double v[1];
    v[0] = sum_pairs(N, pair, [&](long p, double acc, bool two) {
        if (two) {
            const float2 a = *reinterpret_cast<const float2 *>(x + p);
            acc += (double)a.x;
            acc += (double)a.y;
            return acc;
        }
        return acc + (double)x[p];
    });
    block_sum_store<1>(v, partials);
    zero_unused_partials<1>(partials);
}

// phi += e - <e>: the correction, with the zero-mean pin folded in
// (phi is pinned before the step, so <phi + e> = <e>).
__global__ void k_ir_update(double *__restrict__ phi, const float *__restrict__ e, long N,
                            const double *__restrict__ mean)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) phi[p] += (double)e[p] - *mean;
}

// -------------------------------------------------------------------- utility

__global__ void k_fill(double *__restrict__ x, long N, double v)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) x[p] = v;
}

__global__ void k_fill_f32(float *__restrict__ x, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) x[p] = 0.0f;
}

__global__ void k_copy_f32(float *__restrict__ d, const float *__restrict__ s, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = s[p];
}

__global__ void k_copy(double *__restrict__ d, const double *__restrict__ s, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = s[p];
}

__global__ void k_sub_scalar(double *__restrict__ x, long N, const double *__restrict__ s)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) x[p] -= *s;
}

__global__ void k_f32_to_f64(double *__restrict__ d, const float *__restrict__ s, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = (double)s[p];
}

__global__ void k_f64_to_f32(float *__restrict__ d, const double *__restrict__ s, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = (float)s[p];
}

__global__ void k_affine_to_f32(float *__restrict__ d, const double *__restrict__ s, long N, double off, double sc,
                                int acc)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = acc ? (float)((double)d[p] + (s[p] - off) * sc) : (float)((s[p] - off) * sc);
}

__global__ void k_f32_scaled_to_f64(double *__restrict__ d, const float *__restrict__ s, long N, double sc)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = (double)s[p] * sc;
}

__global__ void k_sub_arrays(double *__restrict__ d, const double *__restrict__ a, const double *__restrict__ b,
                             long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = a[p] - b[p];
}

__global__ void k_add_f32_out(double *__restrict__ d, const double *__restrict__ a, const float *__restrict__ e,
                              long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) d[p] = a[p] + (double)e[p];
}

__global__ void k_axpy(double *__restrict__ y, const double *__restrict__ x, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) y[p] += x[p];
}

// One dimension of the cubic guess interpolation: `in` is nx x ny x nz
// (x fastest); the output doubles dimension `dim` (0 = x, 1 = y, 2 = z).  A
// fine centre a quarter coarse cell above coarse centre I takes the 4-point
// Lagrange weights (-7, 105, 35, -5)/128 on I-1..I+2; a quarter below, the
// mirror image (-5, 35, 105, -7)/128 on I-2..I+1 (periodic).
__global__ void k_cubic_pass(const double *__restrict__ in, int nx, int ny, int nz, int dim,
                             double *__restrict__ out)
{
    const int ox = dim == 0 ? 2 * nx : nx, oy = dim == 1 ? 2 * ny : ny, oz = dim == 2 ? 2 * nz : nz;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long)ox * oy * oz) return;
    const int x = (int)(p % ox), y = (int)((p / ox) % oy), z = (int)(p / ((long)ox * oy));
    const int f = dim == 0 ? x : (dim == 1 ? y : z);
    const int nd = dim == 0 ? nx : (dim == 1 ? ny : nz);
    const int I = f >> 1;
    const int first = (f & 1) ? I - 1 : I - 2;
    const double w0 = (f & 1) ? -7.0 : -5.0, w1 = (f & 1) ? 105.0 : 35.0, w2 = (f & 1) ? 35.0 : 105.0,
                 w3 = (f & 1) ? -5.0 : -7.0;
    const long stride = dim == 0 ? 1 : (dim == 1 ? (long)nx : (long)nx * ny);
    const long base = dim == 0 ? ((long)z * ny + y) * nx : (dim == 1 ? (long)z * ny * nx + x : (long)y * nx + x);
    auto at = [&](int k) { return in[base + (long)wrapi(first + k, nd) * stride]; };
    out[p] = (w0 * at(0) + w1 * at(1) + w2 * at(2) + w3 * at(3)) * (1.0 / 128.0);
}

__global__ void k_set_scalar(double *slot, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *slot = v;
}

inline unsigned blocks_for(long count) { return (unsigned)((count + TPB - 1) / TPB); }

// ------------------------------------------------ vectorised elementwise passes
//
// Streaming passes over n^3 arrays move four consecutive elements per thread
// and iteration as 16-byte loads and stores (two double2 or one float4), in a
// grid-stride loop over at most kEwBlocks workgroups, so that every thread keeps
// several wide loads in flight.  Launchers take this form when every pointer is
// 16-byte aligned and fall back to one element per thread otherwise; both forms
// compute each element by the same expression.
constexpr unsigned kEwBlocks = 4096;

struct D4 {
    double2 lo, hi;
};
__device__ __forceinline__ D4 ld4(const double *p)
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
    return D4{q[0], q[1]};
}
__device__ __forceinline__ void st4(double *p, const D4 &v)
{
    double2 *q = reinterpret_cast<double2 *>(p);
    q[0] = v.lo;
    q[1] = v.hi;
}
__device__ __forceinline__ float4 ldf4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void stf4(float *p, const float4 &v) { *reinterpret_cast<float4 *>(p) = v; }

template <class Op>
__global__ void __launch_bounds__(TPB) k_ew4(long groups, Op op)
{
    for (long q = (long)blockIdx.x * TPB + threadIdx.x; q < groups; q += (long)gridDim.x * TPB) op(4 * q);
}

inline bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// launches op over the first N - N % 4 elements; returns the count done
template <class Op>
long launch_ew4(hipStream_t s, long N, Op op)
{
    const long groups = N / 4;
    if (groups <= 0) return 0;
    long b = (groups + TPB - 1) / TPB;
    if (b > (long)kEwBlocks) b = kEwBlocks;
    k_ew4<Op><<<(unsigned)b, TPB, 0, s>>>(groups, op);
    return 4 * groups;
}

struct EwFill {
    double *x;
    double v;
    __device__ void operator()(long p) const { st4(x + p, D4{make_double2(v, v), make_double2(v, v)}); }
};
struct EwCopy {
    double *d;
    const double *a;
    __device__ void operator()(long p) const { st4(d + p, ld4(a + p)); }
};
struct EwSubScalar {
    double *x;
    const double *sc;
    __device__ void operator()(long p) const
    {
        const double c = *sc;
        D4 v = ld4(x + p);
        v.lo.x -= c;
        v.lo.y -= c;
        v.hi.x -= c;
        v.hi.y -= c;
        st4(x + p, v);
    }
};
struct EwSubArrays {
    double *d;
    const double *a, *b;
    __device__ void operator()(long p) const
    {
        const D4 u = ld4(a + p), w = ld4(b + p);
        st4(d + p, D4{make_double2(u.lo.x - w.lo.x, u.lo.y - w.lo.y), make_double2(u.hi.x - w.hi.x, u.hi.y - w.hi.y)});
    }
};
struct EwAxpy {
    double *y;
    const double *x;
    __device__ void operator()(long p) const
    {
        D4 v = ld4(y + p);
        const D4 u = ld4(x + p);
        v.lo.x += u.lo.x;
        v.lo.y += u.lo.y;
        v.hi.x += u.hi.x;
        v.hi.y += u.hi.y;
        st4(y + p, v);
    }
};
struct EwIrUpdate { // phi += e - <e>
    double *phi;
    const float *e;
    const double *mean;
    __device__ void operator()(long p) const
    {
        const double m = *mean;
        D4 v = ld4(phi + p);
        const float4 c = ldf4(e + p);
        v.lo.x += (double)c.x - m;
        v.lo.y += (double)c.y - m;
        v.hi.x += (double)c.z - m;
        v.hi.y += (double)c.w - m;
        st4(phi + p, v);
    }
};
struct EwAddF32Out { // d = a + e
    double *d;
    const double *a;
    const float *e;
    __device__ void operator()(long p) const
    {
        const D4 v = ld4(a + p);
        const float4 c = ldf4(e + p);
        st4(d + p, D4{make_double2(v.lo.x + (double)c.x, v.lo.y + (double)c.y),
                      make_double2(v.hi.x + (double)c.z, v.hi.y + (double)c.w)});
    }
};
struct EwExtrapolate { // history-based guess: see launch_extrapolate
    double *field, *hist, *alt;
    const double *add;
    bool hv;
    __device__ void operator()(long p) const
    {
        const D4 o = ld4(field + p), a = ld4(add + p);
        D4 r;
        if (hv) {
            const D4 h = ld4(hist + p);
            r = D4{make_double2((2.0 * o.lo.x - h.lo.x) + a.lo.x, (2.0 * o.lo.y - h.lo.y) + a.lo.y),
                   make_double2((2.0 * o.hi.x - h.hi.x) + a.hi.x, (2.0 * o.hi.y - h.hi.y) + a.hi.y)};
        } else {
            r = D4{make_double2(o.lo.x + a.lo.x, o.lo.y + a.lo.y), make_double2(o.hi.x + a.hi.x, o.hi.y + a.hi.y)};
        }
        st4(field + p, r);
        st4(hist + p, o);
        st4(alt + p, o);
    }
};
struct EwFillF32 {
    float *x;
    __device__ void operator()(long p) const { stf4(x + p, make_float4(0.f, 0.f, 0.f, 0.f)); }
};
struct EwCopyF32 {
    float *d;
    const float *a;
    __device__ void operator()(long p) const { stf4(d + p, ldf4(a + p)); }
};
struct EwNegToF32 {
    float *d;
    const double *a;
    __device__ void operator()(long p) const
    {
        const D4 v = ld4(a + p);
        stf4(d + p, make_float4((float)(-v.lo.x), (float)(-v.lo.y), (float)(-v.hi.x), (float)(-v.hi.y)));
    }
};
struct EwF32ToF64 {
    double *d;
    const float *a;
    __device__ void operator()(long p) const
    {
        const float4 c = ldf4(a + p);
        st4(d + p, D4{make_double2((double)c.x, (double)c.y), make_double2((double)c.z, (double)c.w)});
    }
};
struct EwF64ToF32 {
    float *d;
    const double *a;
    __device__ void operator()(long p) const
    {
        const D4 v = ld4(a + p);
        stf4(d + p, make_float4((float)v.lo.x, (float)v.lo.y, (float)v.hi.x, (float)v.hi.y));
    }
};

} // namespace

#define GR_DISPATCH_KIND_G(kind, KERNEL, G, ...)                                                      \
    do {                                                                                              \
        if ((kind) == GR_KIND_POISSON) KERNEL<GR_KIND_POISSON><<<(G).grid, (G).block, 0, s>>>(__VA_ARGS__); \
        else if ((kind) == GR_KIND_HAMILTONIAN)                                                       \
            KERNEL<GR_KIND_HAMILTONIAN><<<(G).grid, (G).block, 0, s>>>(__VA_ARGS__);                  \
        else KERNEL<GR_KIND_CMC><<<(G).grid, (G).block, 0, s>>>(__VA_ARGS__);                        \
    } while (0)

// dispatch over all six kinds, with a scalar type T
#define GR_DISPATCH_KT(kind, T, KERNEL, GRID, BLOCK, ...)                                              \
    do {                                                                                              \
        switch (kind) {                                                                               \
        case GR_KIND_POISSON: KERNEL<GR_KIND_POISSON, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;  \
        case GR_KIND_HAMILTONIAN: KERNEL<GR_KIND_HAMILTONIAN, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break; \
        case GR_KIND_CMC: KERNEL<GR_KIND_CMC, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;          \
        case K_LIN_POISSON: KERNEL<K_LIN_POISSON, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;      \
        case K_LIN_HAM: KERNEL<K_LIN_HAM, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;              \
        default: KERNEL<K_LIN_CMC, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;                     \
        }                                                                                             \
    } while (0)

#define GR_DISPATCH_K2T(kind, TG, T, KERNEL, GRID, BLOCK, ...)                                          \
    do {                                                                                              \
        switch (kind) {                                                                               \
        case GR_KIND_POISSON: KERNEL<GR_KIND_POISSON, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break; \
        case GR_KIND_HAMILTONIAN: KERNEL<GR_KIND_HAMILTONIAN, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break; \
        case GR_KIND_CMC: KERNEL<GR_KIND_CMC, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;      \
        case K_LIN_POISSON: KERNEL<K_LIN_POISSON, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;  \
        case K_LIN_HAM: KERNEL<K_LIN_HAM, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;          \
        default: KERNEL<K_LIN_CMC, TG, T><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); break;                 \
        }                                                                                             \
    } while (0)

template <typename T>
void launch_rb_sweep_t(int kind, hipStream_t s, T *phi, const T *f, const T *c1, const T *c2, int n, double h,
                       OpConst oc, const double *fbar, const double *fshift)
{
    const T inv_h2 = T(1.0 / (h * h));
    const Geo G = geo3(n / 2, n, n);
    for (int colour = 0; colour < 2; ++colour)
        GR_DISPATCH_KT(kind, T, k_rb_colour, G.grid, G.block, phi, f, c1, c2, n, inv_h2, colour, oc, fbar, fshift);
}

void launch_rb_sweep(int kind, hipStream_t s, double *phi, const double *f, const double *coef, int n, double h,
                     OpConst oc, const double *fbar, const double *fshift)
{
    launch_rb_sweep_t<double>(kind, s, phi, f, coef, nullptr, n, h, oc, fbar, fshift);
}

void launch_rb_sweep_f32(int kind, hipStream_t s, float *e, const float *b, const float *c1, const float *c2, int n,
                         double h, OpConst oc, const double *zero)
{
    launch_rb_sweep_t<float>(kind, s, e, b, c1, c2, n, h, oc, zero, zero);
}

// 64-wide tiles need n % 64 == 0; levels of n % 64 == 32 (e.g. 32^3) take the 32 x 16 tile
bool fused_sweep_ok(int n, int min_n) { return n >= min_n && n >= 32 && n % 32 == 0; }

template <int KIND, typename T, int TX, int TY>
static void launch_fused_k(int pf, unsigned grid, hipStream_t s, const T *in, T *out, const T *f, const T *c1,
                           const T *c2, int n, int zc, T inv_h2, OpConst oc, const double *fbar,
                           const double *fshift, int tiles_y, int xcd_remap)
{
    constexpr int NT = (TX / 2) * TY;
    // default prefetch depth (measured at 256^3): two planes, except for the
    // FP64 Hamiltonian and CMC sweeps in tiles under 64x16, whose extra
    // registers would cost a resident workgroup per CU
    if (pf <= 0) pf = (TX * TY >= 1024 || sizeof(T) == 4 || KIND == GR_KIND_POISSON) ? 2 : 1;
    // deeper prefetch (3 or 4 planes) is built for the 64 x 16 tile only
    if (pf > 2 && TX * TY < 1024) pf = 2;
    if (TX * TY >= 1024 && pf == 4)
        k_rb_fused<KIND, T, TX, TY, (TX * TY >= 1024 ? 4 : 2)><<<grid, NT, 0, s>>>(
            in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift, tiles_y, xcd_remap);
    else if (TX * TY >= 1024 && pf == 3)
        k_rb_fused<KIND, T, TX, TY, (TX * TY >= 1024 ? 3 : 2)><<<grid, NT, 0, s>>>(
            in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift, tiles_y, xcd_remap);
    else if (pf == 2)
        k_rb_fused<KIND, T, TX, TY, 2><<<grid, NT, 0, s>>>(in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift,
                                                             tiles_y, xcd_remap);
    else
        k_rb_fused<KIND, T, TX, TY, 1><<<grid, NT, 0, s>>>(in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift,
                                                             tiles_y, xcd_remap);
}

template <typename T, int TX, int TY>
static void launch_fused_t(int kind, hipStream_t s, const T *in, T *out, const T *f, const T *c1, const T *c2, int n,
                           double h, OpConst oc, const double *fbar, const double *fshift, const FusedCfg &cfg)
{
    const int tiles_x = n / TX, tiles_y = n / TY;
    const int tiles = tiles_x * tiles_y;
    // z chunk: halve (keeping >= 8 planes, GRMG_FUSED_ZMIN, and a divisor of n)
    // until the grid reaches the target number of workgroups (one resident wave);
    // shorter chunks on the small levels (2 planes) measured no faster in the solve
    static const int zmin = [] {
        const char *e = std::getenv("GRMG_FUSED_ZMIN");
        return e ? std::max(1, std::atoi(e)) : 8;
    }();
    int zc = n;
    while (zc % 2 == 0 && zc / 2 >= zmin && (long)tiles * (n / zc) < cfg.target_wgs) zc /= 2;
    const unsigned grid = (unsigned)(tiles * (n / zc));
    const T inv_h2 = T(1.0 / (h * h));
#define GR_FUSED_CASE(K)                                                                                      \
    case K:                                                                                                   \
        launch_fused_k<K, T, TX, TY>(cfg.pf, grid, s, in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift,    \
                                     tiles_y, cfg.xcd_remap);                                                 \
        break;
    switch (kind) {
        GR_FUSED_CASE(GR_KIND_POISSON)
        GR_FUSED_CASE(GR_KIND_HAMILTONIAN)
        GR_FUSED_CASE(GR_KIND_CMC)
        GR_FUSED_CASE(K_LIN_POISSON)
        GR_FUSED_CASE(K_LIN_HAM)
    default:
        launch_fused_k<K_LIN_CMC, T, TX, TY>(cfg.pf, grid, s, in, out, f, c1, c2, n, zc, inv_h2, oc, fbar, fshift,
                                             tiles_y, cfg.xcd_remap);
        break;
    }
#undef GR_FUSED_CASE
}

template <typename T>
static void launch_fused_any(int kind, hipStream_t s, const T *in, T *out, const T *f, const T *c1, const T *c2,
                             int n, double h, OpConst oc, const double *fbar, const double *fshift, const FusedCfg &cfg)
{
    if (cfg.tile == 1 || n % 64 != 0)
        launch_fused_t<T, 32, 16>(kind, s, in, out, f, c1, c2, n, h, oc, fbar, fshift, cfg);
    else if (cfg.tile == 3 && n % 128 == 0) // 1 KB contiguous rows; other sizes take 64x16
        launch_fused_t<T, 128, 8>(kind, s, in, out, f, c1, c2, n, h, oc, fbar, fshift, cfg);
    else if (cfg.tile >= 2)
        launch_fused_t<T, 64, 16>(kind, s, in, out, f, c1, c2, n, h, oc, fbar, fshift, cfg);
    else
        launch_fused_t<T, 64, 8>(kind, s, in, out, f, c1, c2, n, h, oc, fbar, fshift, cfg);
}

void launch_rb_fused(int kind, hipStream_t s, const double *in, double *out, const double *f, const double *coef,
                     int n, double h, OpConst oc, const double *fbar, const double *fshift, const FusedCfg &cfg)
{
    launch_fused_any<double>(kind, s, in, out, f, coef, nullptr, n, h, oc, fbar, fshift, cfg);
}

void launch_rb_fused_f32(int kind, hipStream_t s, const float *in, float *out, const float *b, const float *c1,
                         const float *c2, int n, double h, OpConst oc, const double *zero, const FusedCfg &cfg)
{
    launch_fused_any<float>(kind, s, in, out, b, c1, c2, n, h, oc, zero, zero, cfg);
}

// Plane-marching kernels serve levels with n a multiple of 32 and n >= 64
// (GRMG_MARCH=0 keeps the one-thread-per-point kernels everywhere).  The z
// chunk is halved (even, >= 8 planes) while the grid stays within max_blocks.
bool march_ok(int n)
{
    static const bool on = [] {
        const char *e = std::getenv("GRMG_MARCH");
        return !(e && std::atoi(e) == 0);
    }();
    return on && n >= 64 && n % MTX == 0;
}

// workgroups of the row-walking norm kernels (4 x-rows each, at most kReduceBlocks)
unsigned row_blocks(int n)
{
    const long b = ((long)n * n + 3) / 4;
    return (unsigned)(b > kReduceBlocks ? kReduceBlocks : b);
}

// Workgroup budget of the plane-marching kernels that also reduce (norms,
// refinement residuals); at most kReduceBlocks.  More workgroups raise the
// occupancy, shorter z-chunks re-read more halo planes.  GRMG_MARCH_BLOCKS
// overrides the default.
long march_norm_blocks()
{
    static const long b = [] {
        long v = 2048;
        if (const char *e = std::getenv("GRMG_MARCH_BLOCKS")) v = std::atol(e);
        return v < 64 ? 64L : (v > kReduceBlocks ? (long)kReduceBlocks : v);
    }();
    return b;
}

// the x-pair form serves levels whose side is a multiple of 64 (GRMG_MARCH2=0: off)
bool march2_ok(int n)
{
    static const bool on = [] {
        const char *e = std::getenv("GRMG_MARCH2");
        return !(e && std::atoi(e) == 0);
    }();
    return on && march_ok(n) && n % M2TX == 0;
}

// Grid of the x-pair passes; *zc_out carries the z-chunk length in its low 16
// bits and the block order in bit 16 (z-chunk major in contiguous runs per XCD,
// taken when the grid is a multiple of 8; GRMG_MARCH2_ORDER=0: tile major).
int march2_grid(int n, long max_blocks, int *zc_out)
{
    static const int order = [] {
        const char *e = std::getenv("GRMG_MARCH2_ORDER");
        return e ? std::atoi(e) : 1;
    }();
    const long tiles = (long)(n / M2TX) * (n / M2TY);
    if (tiles > max_blocks) return 0;
    int zc = n;
    while (zc % 4 == 0 && zc / 2 >= 8 && tiles * (n / (zc / 2)) <= max_blocks) zc /= 2;
    const long grid = tiles * (n / zc);
    *zc_out = zc | ((order == 1 && grid % 8 == 0) ? (1 << 16) : 0);
    return (int)grid;
}

int march_grid(int n, long max_blocks, int *zc_out)
{
    const long tiles = (long)(n / MTX) * (n / MTY);
    if (tiles > max_blocks) return 0;
    int zc = n;
    while (zc % 4 == 0 && zc / 2 >= 8 && tiles * (n / (zc / 2)) <= max_blocks) zc /= 2;
    *zc_out = zc;
    return (int)(tiles * (n / zc));
}

#define GR_MARCH_KIND(MODE, T, kind, grid, ...)                                                       \
    do {                                                                                              \
        switch (kind) {                                                                               \
        case GR_KIND_POISSON: k_march<MODE, GR_KIND_POISSON, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break; \
        case GR_KIND_HAMILTONIAN: k_march<MODE, GR_KIND_HAMILTONIAN, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break; \
        case GR_KIND_CMC: k_march<MODE, GR_KIND_CMC, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break;          \
        case K_LIN_POISSON: k_march<MODE, K_LIN_POISSON, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break;      \
        case K_LIN_HAM: k_march<MODE, K_LIN_HAM, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break;              \
        default: k_march<MODE, K_LIN_CMC, T><<<grid, MNT, 0, s>>>(__VA_ARGS__, nullptr); break;                     \
        }                                                                                             \
    } while (0)

#define GR_MARCH2_KIND(MODE, T, kind, grid, ...)                                                      \
    do {                                                                                              \
        switch (kind) {                                                                               \
        case GR_KIND_POISSON: k_march2<MODE, GR_KIND_POISSON, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break; \
        case GR_KIND_HAMILTONIAN: k_march2<MODE, GR_KIND_HAMILTONIAN, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break; \
        case GR_KIND_CMC: k_march2<MODE, GR_KIND_CMC, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break;          \
        case K_LIN_POISSON: k_march2<MODE, K_LIN_POISSON, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break;      \
        case K_LIN_HAM: k_march2<MODE, K_LIN_HAM, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break;              \
        default: k_march2<MODE, K_LIN_CMC, T><<<grid, M2NT, 0, s>>>(__VA_ARGS__, nullptr); break;                     \
        }                                                                                             \
    } while (0)

void launch_residual_restrict(int kind, hipStream_t s, const double *phi, const double *f, const double *coef,
                              int n, double h, OpConst oc, const double *fbar, const double *fshift,
                              double *phi_c, double *phi0_c, double *rr_c)
{
    int zc = 0, grid = 0;
    if (march2_ok(n) && (grid = march2_grid(n, 4096, &zc)) > 0) {
        const double ih2 = 1.0 / (h * h);
        switch (kind) {
        case GR_KIND_POISSON:
            k_march2<M_RESTRICT, GR_KIND_POISSON, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr, nullptr,
                nullptr, nullptr);
            break;
        case GR_KIND_HAMILTONIAN:
            k_march2<M_RESTRICT, GR_KIND_HAMILTONIAN, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr, nullptr,
                nullptr, nullptr);
            break;
        default:
            k_march2<M_RESTRICT, GR_KIND_CMC, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr, nullptr,
                nullptr, nullptr);
            break;
        }
        return;
    }
    if (march_ok(n) && (grid = march_grid(n, 4096, &zc)) > 0) {
        switch (kind) {
        case GR_KIND_POISSON:
            k_march<M_RESTRICT, GR_KIND_POISSON, double><<<grid, MNT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, 1.0 / (h * h), oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr,
                nullptr, nullptr, nullptr);
            break;
        case GR_KIND_HAMILTONIAN:
            k_march<M_RESTRICT, GR_KIND_HAMILTONIAN, double><<<grid, MNT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, 1.0 / (h * h), oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr,
                nullptr, nullptr, nullptr);
            break;
        default:
            k_march<M_RESTRICT, GR_KIND_CMC, double><<<grid, MNT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, 1.0 / (h * h), oc, fbar, fshift, nullptr, phi_c, phi0_c, rr_c, nullptr,
                nullptr, nullptr, nullptr);
            break;
        }
        return;
    }
    const int m = n / 2;
    GR_DISPATCH_KIND_G(kind, k_residual_restrict, geo3(m, m, m), phi, f, coef, n, 1.0 / (h * h), oc, fbar, fshift,
                       phi_c, phi0_c, rr_c);
}

void launch_lin_residual_restrict_f32(int kind, hipStream_t s, const float *e, const float *b, const float *c1,
                                      const float *c2, int n, double h, OpConst oc, float *b_c, float *e_c)
{
    const float inv_h2 = float(1.0 / (h * h));
    int zc = 0, grid = 0;
    if (march2_ok(n) && (grid = march2_grid(n, 4096, &zc)) > 0) {
        GR_MARCH2_KIND(M_RESTRICT_LIN, float, kind, grid, e, b, c1, c2, n, zc, inv_h2, oc, nullptr, nullptr, nullptr,
                       b_c, e_c, nullptr, nullptr, nullptr, nullptr);
        return;
    }
    if (march_ok(n) && (grid = march_grid(n, 4096, &zc)) > 0) {
        GR_MARCH_KIND(M_RESTRICT_LIN, float, kind, grid, e, b, c1, c2, n, zc, inv_h2, oc, nullptr, nullptr, nullptr,
                      b_c, e_c, nullptr, nullptr, nullptr, nullptr);
        return;
    }
    const int m = n / 2;
    const Geo G = geo3(m, m, m);
    GR_DISPATCH_KT(kind, float, k_lin_residual_restrict, G.grid, G.block, e, b, c1, c2, n, inv_h2, oc, b_c, e_c);
}

void launch_coarse_rhs(int kind, hipStream_t s, const double *phi_c, const double *coef_c, const double *rr_c,
                       int m, double H, OpConst oc, double *f_c)
{
    GR_DISPATCH_KIND_G(kind, k_coarse_rhs, geo3(m, m, m), phi_c, coef_c, rr_c, m, 1.0 / (H * H), oc, f_c);
}

void launch_residual(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                     double h, OpConst oc, const double *fbar, const double *fshift, double *r)
{
    GR_DISPATCH_KIND_G(kind, k_residual, geo3(n, n, n), phi, f, coef, n, 1.0 / (h * h), oc, fbar, fshift, r);
}

void launch_prolong_correct(hipStream_t s, double *phi_f, int n, const double *phi_c, const double *phi0_c)
{
    const ProlongGeo G = prolong_geo(n);
    k_prolong_correct<double, true><<<G.grid, G.block, 0, s>>>(phi_f, n, G.zc, phi_c, phi0_c);
}

void launch_prolong_add_f64(hipStream_t s, double *phi_f, int n, const double *e_c)
{
    const ProlongGeo G = prolong_geo(n);
    k_prolong_correct<double, false><<<G.grid, G.block, 0, s>>>(phi_f, n, G.zc, e_c, nullptr);
}

void launch_sub_arrays(hipStream_t s, double *d, const double *a, const double *b, long N)
{
    const long done = al16(d) && al16(a) && al16(b) ? launch_ew4(s, N, EwSubArrays{d, a, b}) : 0;
    if (N > done) k_sub_arrays<<<blocks_for(N - done), TPB, 0, s>>>(d + done, a + done, b + done, N - done);
}

void launch_prolong_add_f32(hipStream_t s, float *e_f, int n, const float *e_c)
{
    const ProlongGeo G = prolong_geo(n);
    k_prolong_correct<float, false><<<G.grid, G.block, 0, s>>>(e_f, n, G.zc, e_c, nullptr);
}

void launch_restrict(hipStream_t s, const double *fine, int n, double *coarse)
{
    const Geo G = geo3(n / 2, n / 2, n / 2);
    k_restrict<double><<<G.grid, G.block, 0, s>>>(fine, n, coarse);
}

void launch_restrict_f32(hipStream_t s, const float *fine, int n, float *coarse)
{
    const Geo G = geo3(n / 2, n / 2, n / 2);
    k_restrict<float><<<G.grid, G.block, 0, s>>>(fine, n, coarse);
}

template <typename TG, typename T>
static bool coarse_lds_fits(int kind, const CoarseLevelsT<TG> &C)
{
    static const bool on = [] {
        const char *e = std::getenv("GRMG_COARSE_LDS");
        return !(e && std::atoi(e) == 0);
    }();
    if (!on) return false;
    size_t b = 0;
    switch (kind) {
    case GR_KIND_POISSON: b = coarse_lds_layout<GR_KIND_POISSON, TG, T>(C, nullptr, (T *)nullptr); break;
    case GR_KIND_HAMILTONIAN: b = coarse_lds_layout<GR_KIND_HAMILTONIAN, TG, T>(C, nullptr, (T *)nullptr); break;
    case GR_KIND_CMC: b = coarse_lds_layout<GR_KIND_CMC, TG, T>(C, nullptr, (T *)nullptr); break;
    case K_LIN_POISSON: b = coarse_lds_layout<K_LIN_POISSON, TG, T>(C, nullptr, (T *)nullptr); break;
    case K_LIN_HAM: b = coarse_lds_layout<K_LIN_HAM, TG, T>(C, nullptr, (T *)nullptr); break;
    default: b = coarse_lds_layout<K_LIN_CMC, TG, T>(C, nullptr, (T *)nullptr); break;
    }
    return b <= kCoarseLdsBytes;
}

void launch_coarse_vcycle(int kind, hipStream_t s, const CoarseLevelsT<double> &C, int nu1, int nu2, OpConst oc,
                          const double *fbar0, const double *fshift0)
{
    if (coarse_lds_fits<double, double>(kind, C)) {
        GR_DISPATCH_K2T(kind, double, double, k_coarse_vcycle_lds, 1, CTPB, C, nu1, nu2, oc, fbar0, fshift0);
        return;
    }
    GR_DISPATCH_KT(kind, double, k_coarse_vcycle, 1, CTPB, C, nu1, nu2, oc, fbar0, fshift0);
}

void launch_coarse_vcycle_f32(int kind, hipStream_t s, const CoarseLevelsT<float> &C, int nu1, int nu2, OpConst oc,
                              const double *zero)
{
    // FP32 arrays, the cycle in FP64 in LDS (the global-memory fallback, for
    // thresholds whose levels do not fit, computes in FP32)
    if (coarse_lds_fits<float, double>(kind, C)) {
        GR_DISPATCH_K2T(kind, float, double, k_coarse_vcycle_lds, 1, CTPB, C, nu1, nu2, oc, zero, zero);
        return;
    }
    GR_DISPATCH_KT(kind, float, k_coarse_vcycle, 1, CTPB, C, nu1, nu2, oc, zero, zero);
}

void launch_ir_residual(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                        double h, OpConst oc, const double *fbar, const double *fshift, float *b32, float *a32,
                        float *c32, double *partials)
{
    int zc = 0, grid = 0;
    if (march2_ok(n) && (grid = march2_grid(n, march_norm_blocks(), &zc)) > 0) {
        const double ih2 = 1.0 / (h * h);
        if (kind == GR_KIND_POISSON)
            k_march2<M_IR, GR_KIND_POISSON, double><<<grid, M2NT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc,
                                                                         fbar, fshift, partials, nullptr, nullptr,
                                                                         nullptr, b32, a32, c32, nullptr);
        else if (kind == GR_KIND_HAMILTONIAN)
            k_march2<M_IR, GR_KIND_HAMILTONIAN, double><<<grid, M2NT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc,
                                                                             fbar, fshift, partials, nullptr,
                                                                             nullptr, nullptr, b32, a32, c32,
                                                                             nullptr);
        else
            k_march2<M_IR, GR_KIND_CMC, double><<<grid, M2NT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc, fbar,
                                                                     fshift, partials, nullptr, nullptr, nullptr,
                                                                     b32, a32, c32, nullptr);
        return;
    }
    if (march_ok(n) && (grid = march_grid(n, march_norm_blocks(), &zc)) > 0) {
        const double ih2 = 1.0 / (h * h);
        if (kind == GR_KIND_POISSON)
            k_march<M_IR, GR_KIND_POISSON, double><<<grid, MNT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc, fbar,
                                                                       fshift, partials, nullptr, nullptr, nullptr,
                                                                       b32, a32, c32, nullptr);
        else if (kind == GR_KIND_HAMILTONIAN)
            k_march<M_IR, GR_KIND_HAMILTONIAN, double><<<grid, MNT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc,
                                                                           fbar, fshift, partials, nullptr, nullptr,
                                                                           nullptr, b32, a32, c32, nullptr);
        else
            k_march<M_IR, GR_KIND_CMC, double><<<grid, MNT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc, fbar,
                                                                   fshift, partials, nullptr, nullptr, nullptr, b32,
                                                                   a32, c32, nullptr);
        return;
    }
    Geo G;
    G.grid = dim3(row_blocks(n));
    G.block = dim3(64, 4);
    GR_DISPATCH_KIND_G(kind, k_ir_residual, G, phi, f, coef, n, 1.0 / (h * h), oc, fbar, fshift, b32, a32, c32,
                       partials);
}

// phi_out = phi + e and, for phi_out, the Poisson FP64 residual as FP32 b =
// -eps and the stopping norms (one plane-marching pass when the level allows,
// else an update pass and the residual pass)
void launch_ir_update_residual(hipStream_t s, const double *phi, const float *e, double *phi_out, const double *f,
                               int n, double h, OpConst oc, const double *fbar, const double *fshift, float *b32,
                               double *partials)
{
    int zc = 0, grid = 0;
    if (march2_ok(n) && (grid = march2_grid(n, march_norm_blocks(), &zc)) > 0) {
        k_march2<M_IRU, GR_KIND_POISSON, double><<<grid, M2NT, 0, s>>>(phi, f, nullptr, nullptr, n, zc,
                                                                      1.0 / (h * h), oc, fbar, fshift, partials,
                                                                      phi_out, nullptr, nullptr, b32, nullptr,
                                                                      nullptr, e);
        return;
    }
    if (march_ok(n) && (grid = march_grid(n, march_norm_blocks(), &zc)) > 0) {
        k_march<M_IRU, GR_KIND_POISSON, double><<<grid, MNT, 0, s>>>(phi, f, nullptr, nullptr, n, zc, 1.0 / (h * h),
                                                                    oc, fbar, fshift, partials, phi_out, nullptr,
                                                                    nullptr, b32, nullptr, nullptr, e);
        return;
    }
    const long N = (long)n * n * n;
    const long done = al16(phi_out) && al16(phi) && al16(e) ? launch_ew4(s, N, EwAddF32Out{phi_out, phi, e}) : 0;
    if (N > done) k_add_f32_out<<<blocks_for(N - done), TPB, 0, s>>>(phi_out + done, phi + done, e + done, N - done);
    launch_ir_residual(GR_KIND_POISSON, s, phi_out, f, nullptr, n, h, oc, fbar, fshift, b32, nullptr, nullptr,
                       partials);
}

void launch_neg_to_f32(hipStream_t s, float *dst, const double *src, long N)
{
    const long done = al16(dst) && al16(src) ? launch_ew4(s, N, EwNegToF32{dst, src}) : 0;
    if (N > done) k_neg_to_f32<<<blocks_for(N - done), TPB, 0, s>>>(dst + done, src + done, N - done);
}

void launch_sum_f32(hipStream_t s, const float *x, long N, double *partials)
{
    k_sum_f32<<<reduce_blocks(N), TPB, 0, s>>>(x, N, N % 2 == 0 && (reinterpret_cast<uintptr_t>(x) & 7) == 0,
                                               partials);
}

void launch_ir_update(hipStream_t s, double *phi, const float *e, long N, const double *mean)
{
    const long done = al16(phi) && al16(e) ? launch_ew4(s, N, EwIrUpdate{phi, e, mean}) : 0;
    if (N > done) k_ir_update<<<blocks_for(N - done), TPB, 0, s>>>(phi + done, e + done, N - done, mean);
}

void launch_fill_f32(hipStream_t s, float *x, long N)
{
    const long done = al16(x) ? launch_ew4(s, N, EwFillF32{x}) : 0;
    if (N > done) k_fill_f32<<<blocks_for(N - done), TPB, 0, s>>>(x + done, N - done);
}

void launch_sum(hipStream_t s, const double *x, const double *y, long N, double *partials)
{
    k_sum<<<reduce_blocks(N), TPB, 0, s>>>(x, y, N, N % 2 == 0 && al16(x) && (!y || al16(y)), partials);
}

void launch_sum_prod(hipStream_t s, const double *x, const double *y, long N, double *partials)
{
    k_sum_prod<<<reduce_blocks(N), TPB, 0, s>>>(x, y, N, N % 2 == 0 && al16(x) && al16(y), partials);
}

void launch_sum_ham_F(hipStream_t s, const double *psi, const double *f, const double *coef, long N, OpConst oc,
                      double *partials)
{
    k_sum_ham_F<<<reduce_blocks(N), TPB, 0, s>>>(psi, f, coef, N, oc,
                                                 N % 2 == 0 && al16(psi) && al16(f) && al16(coef), partials);
}

void launch_ir_update_sum(int kind, hipStream_t s, double *phi, const float *e, const double *mean, const double *f,
                          const double *coef, long N, OpConst oc, double *partials)
{
    const bool pair = N % 2 == 0 && al16(phi) && al16(f) && al16(coef) && (reinterpret_cast<uintptr_t>(e) & 7) == 0;
    if (kind == GR_KIND_HAMILTONIAN)
        k_ir_update_sum<true><<<reduce_blocks(N), TPB, 0, s>>>(phi, e, mean, f, coef, N, oc, pair, partials);
    else
        k_ir_update_sum<false><<<reduce_blocks(N), TPB, 0, s>>>(phi, e, mean, f, coef, N, oc, pair, partials);
}

void launch_restrict2_f32(hipStream_t s, const float *fa, const float *fc, int n, float *ca, float *cc)
{
    const Geo G = geo3(n / 2, n / 2, n / 2);
    k_restrict2<<<G.grid, G.block, 0, s>>>(fa, fc, n, ca, cc);
}

void launch_restrict2_chain(hipStream_t s, const RestrictChain &R)
{
    k_restrict2_chain<<<1, kCoarseThreads, 0, s>>>(R);
}

void launch_res_norms(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                      double h, OpConst oc, const double *fbar, const double *fshift, double *partials)
{
    int zc = 0, grid = 0;
    if (march2_ok(n) && (grid = march2_grid(n, march_norm_blocks(), &zc)) > 0) {
        const double ih2 = 1.0 / (h * h);
        if (kind == GR_KIND_POISSON)
            k_march2<M_NORMS, GR_KIND_POISSON, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, partials, nullptr, nullptr, nullptr, nullptr,
                nullptr, nullptr, nullptr);
        else if (kind == GR_KIND_HAMILTONIAN)
            k_march2<M_NORMS, GR_KIND_HAMILTONIAN, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, partials, nullptr, nullptr, nullptr, nullptr,
                nullptr, nullptr, nullptr);
        else
            k_march2<M_NORMS, GR_KIND_CMC, double><<<grid, M2NT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, partials, nullptr, nullptr, nullptr, nullptr,
                nullptr, nullptr, nullptr);
        return;
    }
    if (march_ok(n) && (grid = march_grid(n, march_norm_blocks(), &zc)) > 0) {
        const double ih2 = 1.0 / (h * h);
        if (kind == GR_KIND_POISSON)
            k_march<M_NORMS, GR_KIND_POISSON, double><<<grid, MNT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc, fbar,
                                                                          fshift, partials, nullptr, nullptr,
                                                                          nullptr, nullptr, nullptr, nullptr, nullptr);
        else if (kind == GR_KIND_HAMILTONIAN)
            k_march<M_NORMS, GR_KIND_HAMILTONIAN, double><<<grid, MNT, 0, s>>>(
                phi, f, coef, nullptr, n, zc, ih2, oc, fbar, fshift, partials, nullptr, nullptr, nullptr, nullptr,
                nullptr, nullptr, nullptr);
        else
            k_march<M_NORMS, GR_KIND_CMC, double><<<grid, MNT, 0, s>>>(phi, f, coef, nullptr, n, zc, ih2, oc, fbar,
                                                                      fshift, partials, nullptr, nullptr, nullptr,
                                                                      nullptr, nullptr, nullptr, nullptr);
        return;
    }
    Geo G;
    G.grid = dim3(row_blocks(n));
    G.block = dim3(64, 4);
    GR_DISPATCH_KIND_G(kind, k_res_norms, G, phi, f, coef, n, 1.0 / (h * h), oc, fbar, fshift, partials);
}

void launch_finalize(hipStream_t s, const double *partials, int ncomp, double scale, const double *add, double *out,
                     double *host_out)
{
    static_assert(kReduceBlocks % TPB == 0, "partial slots per thread");
    k_finalize<<<1, TPB, 0, s>>>(partials, ncomp, scale, add, out, host_out);
}

void launch_fill(hipStream_t s, double *x, long N, double v)
{
    const long done = al16(x) ? launch_ew4(s, N, EwFill{x, v}) : 0;
    if (N > done) k_fill<<<blocks_for(N - done), TPB, 0, s>>>(x + done, N - done, v);
}

void launch_copy(hipStream_t s, double *dst, const double *src, long N)
{
    const long done = al16(dst) && al16(src) ? launch_ew4(s, N, EwCopy{dst, src}) : 0;
    if (N > done) k_copy<<<blocks_for(N - done), TPB, 0, s>>>(dst + done, src + done, N - done);
}

void launch_copy_f32(hipStream_t s, float *dst, const float *src, long N)
{
    const long done = al16(dst) && al16(src) ? launch_ew4(s, N, EwCopyF32{dst, src}) : 0;
    if (N > done) k_copy_f32<<<blocks_for(N - done), TPB, 0, s>>>(dst + done, src + done, N - done);
}

void launch_sub_scalar(hipStream_t s, double *x, long N, const double *scal)
{
    const long done = al16(x) ? launch_ew4(s, N, EwSubScalar{x, scal}) : 0;
    if (N > done) k_sub_scalar<<<blocks_for(N - done), TPB, 0, s>>>(x + done, N - done, scal);
}

void launch_convert_f32_to_f64(hipStream_t s, double *dst, const float *src, long N)
{
    const long done = al16(dst) && al16(src) ? launch_ew4(s, N, EwF32ToF64{dst, src}) : 0;
    if (N > done) k_f32_to_f64<<<blocks_for(N - done), TPB, 0, s>>>(dst + done, src + done, N - done);
}

void launch_convert_f64_to_f32(hipStream_t s, float *dst, const double *src, long N)
{
    const long done = al16(dst) && al16(src) ? launch_ew4(s, N, EwF64ToF32{dst, src}) : 0;
    if (N > done) k_f64_to_f32<<<blocks_for(N - done), TPB, 0, s>>>(dst + done, src + done, N - done);
}

void launch_set_scalar(hipStream_t s, double *slot, double v) { k_set_scalar<<<1, 64, 0, s>>>(slot, v); }

void launch_affine_to_f32(hipStream_t s, float *dst, const double *src, long N, double off, double scale, bool acc)
{
    if (N > 0) k_affine_to_f32<<<blocks_for(N), TPB, 0, s>>>(dst, src, N, off, scale, acc ? 1 : 0);
}

void launch_f32_scaled_to_f64(hipStream_t s, double *dst, const float *src, long N, double scale)
{
    if (N > 0) k_f32_scaled_to_f64<<<blocks_for(N), TPB, 0, s>>>(dst, src, N, scale);
}

void launch_cubic_pass(hipStream_t s, const double *in, int nx, int ny, int nz, int dim, double *out)
{
    const long M = 2L * nx * ny * nz;
    if (M > 0) k_cubic_pass<<<blocks_for(M), TPB, 0, s>>>(in, nx, ny, nz, dim, out);
}

__global__ void k_extrapolate(double *__restrict__ field, double *__restrict__ hist, double *__restrict__ alt,
                              const double *__restrict__ add, bool hv, long N)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const double o = field[p];
    field[p] = (hv ? 2.0 * o - hist[p] : o) + add[p];
    hist[p] = o;
    alt[p] = o;
}

void launch_extrapolate(hipStream_t s, double *field, double *hist, double *alt, const double *add, bool hv, long N)
{
    const long done = al16(field) && al16(hist) && al16(alt) && al16(add)
                          ? launch_ew4(s, N, EwExtrapolate{field, hist, alt, add, hv})
                          : 0;
    if (N > done)
        k_extrapolate<<<blocks_for(N - done), TPB, 0, s>>>(field + done, hist + done, alt + done, add + done, hv,
                                                           N - done);
}

void launch_axpy(hipStream_t s, double *y, const double *x, long N)
{
    const long done = al16(y) && al16(x) ? launch_ew4(s, N, EwAxpy{y, x}) : 0;
    if (N > done) k_axpy<<<blocks_for(N - done), TPB, 0, s>>>(y + done, x + done, N - done);
}

} // namespace grmg
