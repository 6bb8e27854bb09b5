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
#include "gr_internal.h"

namespace grmg {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ long lin(int i, int j, int k, int n) { return ((long)k * n + j) * n + i; }

// Sum of the six face neighbours of (i,j,k) with periodic wrap.
__device__ __forceinline__ double nb_sum(const double *__restrict__ p, int i, int j, int k, int n)
{
    int ip = wrapi(i + 1, n), im = wrapi(i - 1, n);
    int jp = wrapi(j + 1, n), jm = wrapi(j - 1, n);
    int kp = wrapi(k + 1, n), km = wrapi(k - 1, n);
    return p[lin(ip, j, k, n)] + p[lin(im, j, k, n)] + p[lin(i, jp, k, n)] + p[lin(i, jm, k, n)]
         + p[lin(i, j, kp, n)] + p[lin(i, j, km, n)];
}

// L(phi) at a point (without the source) and dL/dphi there.
template <int KIND>
__device__ __forceinline__ double op_point(double ph, double nbs, double inv_h2, double coef, OpConst oc,
                                           double Fbar, double &J)
{
    const double lap = (nbs - 6.0 * ph) * inv_h2;
    if constexpr (KIND == GR_KIND_POISSON) {
        J = -6.0 * inv_h2;
        return lap;
    } else if constexpr (KIND == GR_KIND_CMC) {
        J = -6.0 * inv_h2 - coef;
        return lap - coef * ph;
    } else {
        const double kap = oc.kappa, A = oc.A;
        const double chi = 1.0 - kap * ph;
        const double chi2 = chi * chi;
        const double chi5 = chi2 * chi2 * chi;
        const double chi6 = chi5 * chi;
        const double chim6 = 1.0 / chi6;
        const double chim7 = chim6 / chi;
        J = -kap * lap - 6.0 * chi * inv_h2 - 6.0 * A * kap * chi5 - 1.5 * kap * coef * chim7 - kap * Fbar;
        return chi * lap + A * (chi6 - 1.0) - 0.25 * coef * chim6 + Fbar * chi;
    }
}

// ----------------------------------------------------------------- smoother

// One colour of a red-black sweep; one thread per point of that colour.
// Colour c holds (i+j+k) % 2 == c; x is split so that consecutive threads
// take consecutive same-colour points of one x-row.
template <int KIND>
__global__ void __launch_bounds__(TPB) k_rb_colour(double *__restrict__ phi, const double *__restrict__ f,
                                                   const double *__restrict__ coef, int n, double inv_h2,
                                                   int colour, OpConst oc, const double *__restrict__ fbar,
                                                   const double *__restrict__ fshift)
{
    const int half = n >> 1;
    const long total = (long)n * n * half;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int i2 = (int)(t % half);
    const long r = t / half;
    const int j = (int)(r % n);
    const int k = (int)(r / n);
    const int i = 2 * i2 + ((j + k + colour) & 1);
    const long p = lin(i, j, k, n);
    const double Fb = *fbar, fs = *fshift;
    const double ph = phi[p];
    double J;
    const double L = op_point<KIND>(ph, nb_sum(phi, i, j, k, n), inv_h2,
                                    KIND == GR_KIND_POISSON ? 0.0 : coef[p], oc, Fb, J);
    phi[p] = ph - (L - (f[p] - fs)) / J;
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
    const long M = (long)m * m * m;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int I = (int)(q % m), J = (int)((q / m) % m), K = (int)(q / ((long)m * m));
    const double Fb = *fbar, fs = *fshift;
    double sr = 0.0, sp = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
        const long p = lin(i, j, k, n);
        const double ph = phi[p];
        double Jd;
        const double L = op_point<KIND>(ph, nb_sum(phi, i, j, k, n), inv_h2,
                                        KIND == GR_KIND_POISSON ? 0.0 : coef[p], oc, Fb, Jd);
        sr += L - (f[p] - fs);
        sp += ph;
    }
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
    const long M = (long)m * m * m;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int I = (int)(q % m), J = (int)((q / m) % m), K = (int)(q / ((long)m * m));
    double Jd;
    const double L = op_point<KIND>(phi_c[q], nb_sum(phi_c, I, J, K, m), inv_H2,
                                    KIND == GR_KIND_POISSON ? 0.0 : coef_c[q], oc, 0.0, Jd);
    f_c[q] = L - rr_c[q];
}

// Residual of one level into r (used by the step-by-step entry point).
template <int KIND>
__global__ void __launch_bounds__(TPB) k_residual(const double *__restrict__ phi, const double *__restrict__ f,
                                                  const double *__restrict__ coef, int n, double inv_h2,
                                                  OpConst oc, const double *__restrict__ fbar,
                                                  const double *__restrict__ fshift, double *__restrict__ r)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    double Jd;
    const double L = op_point<KIND>(phi[p], nb_sum(phi, i, j, k, n), inv_h2,
                                    KIND == GR_KIND_POISSON ? 0.0 : coef[p], oc, *fbar, Jd);
    r[p] = L - (f[p] - *fshift);
}

// Restriction of an arbitrary array: mean of the 8 children.
__global__ void __launch_bounds__(TPB) k_restrict(const double *__restrict__ fine, int n,
                                                  double *__restrict__ coarse)
{
    const int m = n >> 1;
    const long M = (long)m * m * m;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int I = (int)(q % m), J = (int)((q / m) % m), K = (int)(q / ((long)m * m));
    double s = 0.0;
    for (int c = 0; c < 8; ++c)
        s += fine[lin(2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2), n)];
    coarse[q] = s / 8.0;
}

// Cell-centred trilinear prolongation of the coarse correction, added in
// place: fine cell 2I takes 3/4 of coarse cell I and 1/4 of I-1, fine cell
// 2I+1 takes 3/4 of I and 1/4 of I+1 (per axis, periodic).
__global__ void __launch_bounds__(TPB) k_prolong_correct(double *__restrict__ phi_f, int n,
                                                         const double *__restrict__ phi_c,
                                                         const double *__restrict__ phi0_c)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int m = n >> 1;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int I2 = wrapi(I + ((i & 1) ? 1 : -1), m);
    const int J2 = wrapi(J + ((j & 1) ? 1 : -1), m);
    const int K2 = wrapi(K + ((k & 1) ? 1 : -1), m);
    const int Is[2] = {I, I2}, Js[2] = {J, J2}, Ks[2] = {K, K2};
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
        const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
        const long q = lin(Is[ox], Js[oy], Ks[oz], m);
        v += w * (phi_c[q] - phi0_c[q]);
    }
    phi_f[p] += v;
}

// ----------------------------------------------------------------- reductions

// Block-level sum of NC values per thread, fixed order: wavefront shuffles
// (64 lanes) then the waves of the block in order.
template <int NC>
__device__ __forceinline__ void block_sum_store(double (&v)[NC], double *__restrict__ partials)
{
    __shared__ double sh[NC][TPB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = v[c];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[c][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double s = 0.0;
            for (int w = 0; w < TPB / 64; ++w) s += sh[c][w];
            partials[c * kReduceBlocks + blockIdx.x] = s;
        }
    }
}

__global__ void __launch_bounds__(TPB) k_sum(const double *__restrict__ x, const double *__restrict__ y, long N,
                                             double *__restrict__ partials)
{
    double v[1] = {0.0};
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < N; p += (long)kReduceBlocks * TPB)
        v[0] += y ? (x[p] - y[p]) : x[p];
    block_sum_store<1>(v, partials);
}

__global__ void __launch_bounds__(TPB) k_sum_prod(const double *__restrict__ x, const double *__restrict__ y,
                                                  long N, double *__restrict__ partials)
{
    double v[1] = {0.0};
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < N; p += (long)kReduceBlocks * TPB)
        v[0] += x[p] * y[p];
    block_sum_store<1>(v, partials);
}

// Sum of F = (f - A(chi^6 - 1))/chi + AA chi^-7/4 (Hamiltonian regulariser).
__global__ void __launch_bounds__(TPB) k_sum_ham_F(const double *__restrict__ psi, const double *__restrict__ f,
                                                   const double *__restrict__ coef, long N, OpConst oc,
                                                   double *__restrict__ partials)
{
    double v[1] = {0.0};
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < N; p += (long)kReduceBlocks * TPB) {
        const double chi = 1.0 - oc.kappa * psi[p];
        const double chi2 = chi * chi;
        const double chi6 = chi2 * chi2 * chi2;
        const double chim7 = 1.0 / (chi6 * chi);
        v[0] += (f[p] - oc.A * (chi6 - 1.0)) / chi + 0.25 * coef[p] * chim7;
    }
    block_sum_store<1>(v, partials);
}

// Sums of eps^2 and (f - fshift)^2 on one level.
template <int KIND>
__global__ void __launch_bounds__(TPB) k_res_norms(const double *__restrict__ phi, const double *__restrict__ f,
                                                   const double *__restrict__ coef, int n, double inv_h2,
                                                   OpConst oc, const double *__restrict__ fbar,
                                                   const double *__restrict__ fshift,
                                                   double *__restrict__ partials)
{
    const long N = (long)n * n * n;
    const double Fb = *fbar, fs = *fshift;
    double v[2] = {0.0, 0.0};
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < N; p += (long)kReduceBlocks * TPB) {
        const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
        double Jd;
        const double L = op_point<KIND>(phi[p], nb_sum(phi, i, j, k, n), inv_h2,
                                        KIND == GR_KIND_POISSON ? 0.0 : coef[p], oc, Fb, Jd);
        const double fe = f[p] - fs;
        const double e = L - fe;
        v[0] += e * e;
        v[1] += fe * fe;
    }
    block_sum_store<2>(v, partials);
}

// out[c] = (add ? add[c] : 0) + scale * sum of partials of component c, in a
// fixed order (one block; thread t sums blocks t, t+256, ... then a tree).
__global__ void __launch_bounds__(TPB) k_finalize(const double *__restrict__ partials, int ncomp, double scale,
                                                  const double *__restrict__ add, double *__restrict__ out)
{
    __shared__ double sh[TPB];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int b = threadIdx.x; b < kReduceBlocks; b += TPB) s += partials[c * kReduceBlocks + b];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[c] = (add ? add[c] : 0.0) + scale * sh[0];
        __syncthreads();
    }
}

// -------------------------------------------------------------------- utility

__global__ void k_fill(double *__restrict__ x, long N, double v)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) x[p] = v;
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

__global__ void k_set_scalar(double *slot, double v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *slot = v;
}

inline unsigned blocks_for(long count) { return (unsigned)((count + TPB - 1) / TPB); }

} // namespace

#define GR_DISPATCH_KIND(kind, KERNEL, grid, ...)                                                     \
    do {                                                                                              \
        if ((kind) == GR_KIND_POISSON) KERNEL<GR_KIND_POISSON><<<grid, TPB, 0, s>>>(__VA_ARGS__);     \
        else if ((kind) == GR_KIND_HAMILTONIAN) KERNEL<GR_KIND_HAMILTONIAN><<<grid, TPB, 0, s>>>(__VA_ARGS__); \
        else KERNEL<GR_KIND_CMC><<<grid, TPB, 0, s>>>(__VA_ARGS__);                                  \
    } while (0)

void launch_rb_sweep(int kind, hipStream_t s, double *phi, const double *f, const double *coef, int n, double h,
                     OpConst oc, const double *fbar, const double *fshift)
{
    const double inv_h2 = 1.0 / (h * h);
    const unsigned g = blocks_for((long)n * n * (n / 2));
    for (int colour = 0; colour < 2; ++colour)
        GR_DISPATCH_KIND(kind, k_rb_colour, g, phi, f, coef, n, inv_h2, colour, oc, fbar, fshift);
}

void launch_residual_restrict(int kind, hipStream_t s, const double *phi, const double *f, const double *coef,
                              int n, double h, OpConst oc, const double *fbar, const double *fshift,
                              double *phi_c, double *phi0_c, double *rr_c)
{
    const long m = n / 2;
    GR_DISPATCH_KIND(kind, k_residual_restrict, blocks_for(m * m * m), phi, f, coef, n, 1.0 / (h * h), oc, fbar,
                     fshift, phi_c, phi0_c, rr_c);
}

void launch_coarse_rhs(int kind, hipStream_t s, const double *phi_c, const double *coef_c, const double *rr_c,
                       int m, double H, OpConst oc, double *f_c)
{
    GR_DISPATCH_KIND(kind, k_coarse_rhs, blocks_for((long)m * m * m), phi_c, coef_c, rr_c, m, 1.0 / (H * H), oc,
                     f_c);
}

void launch_residual(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                     double h, OpConst oc, const double *fbar, const double *fshift, double *r)
{
    GR_DISPATCH_KIND(kind, k_residual, blocks_for((long)n * n * n), phi, f, coef, n, 1.0 / (h * h), oc, fbar,
                     fshift, r);
}

void launch_prolong_correct(hipStream_t s, double *phi_f, int n, const double *phi_c, const double *phi0_c)
{
    k_prolong_correct<<<blocks_for((long)n * n * n), TPB, 0, s>>>(phi_f, n, phi_c, phi0_c);
}

void launch_restrict(hipStream_t s, const double *fine, int n, double *coarse)
{
    const long m = n / 2;
    k_restrict<<<blocks_for(m * m * m), TPB, 0, s>>>(fine, n, coarse);
}

void launch_sum(hipStream_t s, const double *x, const double *y, long N, double *partials)
{
    k_sum<<<kReduceBlocks, TPB, 0, s>>>(x, y, N, partials);
}

void launch_sum_prod(hipStream_t s, const double *x, const double *y, long N, double *partials)
{
    k_sum_prod<<<kReduceBlocks, TPB, 0, s>>>(x, y, N, partials);
}

void launch_sum_ham_F(hipStream_t s, const double *psi, const double *f, const double *coef, long N, OpConst oc,
                      double *partials)
{
    k_sum_ham_F<<<kReduceBlocks, TPB, 0, s>>>(psi, f, coef, N, oc, partials);
}

void launch_res_norms(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                      double h, OpConst oc, const double *fbar, const double *fshift, double *partials)
{
    GR_DISPATCH_KIND(kind, k_res_norms, kReduceBlocks, phi, f, coef, n, 1.0 / (h * h), oc, fbar, fshift,
                     partials);
}

void launch_finalize(hipStream_t s, const double *partials, int ncomp, double scale, const double *add, double *out)
{
    k_finalize<<<1, TPB, 0, s>>>(partials, ncomp, scale, add, out);
}

void launch_fill(hipStream_t s, double *x, long N, double v)
{
    if (N > 0) k_fill<<<blocks_for(N), TPB, 0, s>>>(x, N, v);
}

void launch_copy(hipStream_t s, double *dst, const double *src, long N)
{
    if (N > 0) k_copy<<<blocks_for(N), TPB, 0, s>>>(dst, src, N);
}

void launch_sub_scalar(hipStream_t s, double *x, long N, const double *scal)
{
    if (N > 0) k_sub_scalar<<<blocks_for(N), TPB, 0, s>>>(x, N, scal);
}

void launch_convert_f32_to_f64(hipStream_t s, double *dst, const float *src, long N)
{
    if (N > 0) k_f32_to_f64<<<blocks_for(N), TPB, 0, s>>>(dst, src, N);
}

void launch_convert_f64_to_f32(hipStream_t s, float *dst, const double *src, long N)
{
    if (N > 0) k_f64_to_f32<<<blocks_for(N), TPB, 0, s>>>(dst, src, N);
}

void launch_set_scalar(hipStream_t s, double *slot, double v) { k_set_scalar<<<1, 64, 0, s>>>(slot, v); }

} // namespace grmg
