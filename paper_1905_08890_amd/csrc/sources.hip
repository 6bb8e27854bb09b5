// Source and coefficient builders for the ten field equations, the CIC
// matter deposit, and the derived fields (paper sec. 4.1.2, 4.3, 4.5).
#include "sources_ops.h"

namespace grmg {

namespace {

constexpr int TPB = 256;
using namespace detail;

__device__ __forceinline__ int wrap_any(long i, int n)
{
    long r = i % n;
    return (int)(r < 0 ? r + n : r);
}

// ------------------------------------------------------------------- CIC

// One thread per particle.  Cell-centred CIC: g = x/h - 1/2, i0 = floor(g),
// t = g - i0, weights (1-t, t) on cells (i0, i0+1), periodic.  chi at the
// particle from the CIC-interpolated Psi; W^2 = c^2 + a^-2 chi^-4 u.u.
__global__ void __launch_bounds__(TPB) k_cic(int n, double a, double c, double kap, const double *__restrict__ pos,
                                             const double *__restrict__ u, double mass, long np,
                                             const double *__restrict__ psi, double *__restrict__ s0,
                                             double *__restrict__ sx, double *__restrict__ sy,
                                             double *__restrict__ sz, double *__restrict__ sm)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    const double h = 1.0 / n;
    int i0[3], i1[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        const double g = pos[3 * q + d] * n - 0.5;
        const double fl = floor(g);
        t[d] = g - fl;
        // fl is finite for finite positions; wrap_any keeps any index in range
        const long il = isfinite(fl) ? (long)fl : 0;
        i0[d] = wrap_any(il, n);
        i1[d] = wrap_any(il + 1, n);
    }
    double psi_p = 0.0;
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        const double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        psi_p += w * psi[lin(ox ? i1[0] : i0[0], oy ? i1[1] : i0[1], oz ? i1[2] : i0[2], n)];
    }
    const double chi = 1.0 - kap * psi_p;
    const double chi2 = chi * chi;
    const double ux = u[3 * q], uy = u[3 * q + 1], uz = u[3 * q + 2];
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double g_uu = u2 / (a * a * chi2 * chi2); // gamma^ij u_i u_j
    const double W = sqrt(c * c + g_uu);
    const double vol = h * h * h;
    const double q0 = mass * W / (c * vol);
    const double qx = mass * ux / (c * vol);
    const double qy = mass * uy / (c * vol);
    const double qz = mass * uz / (c * vol);
    const double qm = mass * g_uu / (W * c * vol); // stress trace gamma^ij s_ij
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        const double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        const long p = lin(ox ? i1[0] : i0[0], oy ? i1[1] : i0[1], oz ? i1[2] : i0[2], n);
        unsafeAtomicAdd(s0 + p, w * q0);
        unsafeAtomicAdd(sx + p, w * qx);
        unsafeAtomicAdd(sy + p, w * qy);
        unsafeAtomicAdd(sz + p, w * qz);
        unsafeAtomicAdd(sm + p, w * qm);
    }
}

// Cell-ordered deposit (no floating-point atomics).  The lower-corner cell of
// each particle's cloud is its key; particles are counted per key, the counts
// are scanned into cell offsets, and each particle writes its weights and
// charges (the per-particle part of the deposit above) to its cell's range.
// Every grid point then sums, in a fixed loop order, the particles of the
// 8 cells whose clouds reach it: the same sums as the scatter, one store per
// point.

struct CicItem {
    double t[3];   // fractional offsets from the lower corner
    double q[5];   // s0, sx, sy, sz, sm charges (before the cloud weights)
};

__device__ __forceinline__ int cic_key(const double *__restrict__ pos, long q, int n, int *i0, double *t)
{
    for (int d = 0; d < 3; ++d) {
        const double g = pos[3 * q + d] * n - 0.5;
        const double fl = floor(g);
        t[d] = g - fl;
        const long il = isfinite(fl) ? (long)fl : 0;
        i0[d] = wrap_any(il, n);
    }
    return (int)lin(i0[0], i0[1], i0[2], n);
}

__global__ void __launch_bounds__(TPB) k_cic_count(int n, const double *__restrict__ pos, long np,
                                                   int *__restrict__ key, int *__restrict__ cnt)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    int i0[3];
    double t[3];
    const int k = cic_key(pos, q, n, i0, t);
    key[q] = k;
    atomicAdd(cnt + k, 1);
}

// Exclusive scan of cnt[0..N) into start[0..N], start[N] = total.  Three
// passes: per-block scan of 2048 items (8 per thread), a one-block scan of
// the block totals, and the block offsets added.
constexpr int kScanItems = 8;
constexpr int kScanTile = TPB * kScanItems;

__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[TPB / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < TPB / 64; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ void __launch_bounds__(TPB) k_scan_tiles(const int *__restrict__ cnt, long N, int *__restrict__ start,
                                                    int *__restrict__ tile_sum)
{
    const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
    int v[kScanItems], sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < N ? cnt[base + i] : 0;
        sum += v[i];
    }
    int total;
    int run = block_excl_scan(sum, &total);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < N) start[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(TPB) k_scan_tile_sums(int *__restrict__ tile_sum, int ntiles,
                                                        int *__restrict__ start_end)
{
    int carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += TPB) {
        const int i = b0 + threadIdx.x;
        const int v = i < ntiles ? tile_sum[i] : 0;
        int total;
        const int ex = block_excl_scan(v, &total);
        if (i < ntiles) tile_sum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *start_end = carry;
}

__global__ void __launch_bounds__(TPB) k_scan_add(int *__restrict__ start, long N, const int *__restrict__ tile_sum,
                                                  int *__restrict__ cur)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    start[p] += tile_sum[p / kScanTile];
    cur[p] = 0;
}

__global__ void __launch_bounds__(TPB) k_cic_place(int n, double a, double c, double kap,
                                                   const double *__restrict__ pos, const double *__restrict__ u,
                                                   double mass, long np, const double *__restrict__ psi,
                                                   const int *__restrict__ key, const int *__restrict__ start,
                                                   int *__restrict__ cur, CicItem *__restrict__ items)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    const double h = 1.0 / n;
    int i0[3], i1[3];
    double t[3];
    cic_key(pos, q, n, i0, t);
    for (int d = 0; d < 3; ++d) i1[d] = i0[d] + 1 == n ? 0 : i0[d] + 1;
    double psi_p = 0.0;
    for (int cc = 0; cc < 8; ++cc) {
        const int ox = cc & 1, oy = (cc >> 1) & 1, oz = cc >> 2;
        const double w = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
        psi_p += w * psi[lin(ox ? i1[0] : i0[0], oy ? i1[1] : i0[1], oz ? i1[2] : i0[2], n)];
    }
    const double chi = 1.0 - kap * psi_p;
    const double chi2 = chi * chi;
    const double ux = u[3 * q], uy = u[3 * q + 1], uz = u[3 * q + 2];
    const double g_uu = (ux * ux + uy * uy + uz * uz) / (a * a * chi2 * chi2);
    const double W = sqrt(c * c + g_uu);
    const double vol = h * h * h;
    const int k = key[q];
    CicItem it;
    it.t[0] = t[0];
    it.t[1] = t[1];
    it.t[2] = t[2];
    it.q[0] = mass * W / (c * vol);
    it.q[1] = mass * ux / (c * vol);
    it.q[2] = mass * uy / (c * vol);
    it.q[3] = mass * uz / (c * vol);
    it.q[4] = mass * g_uu / (W * c * vol);
    items[start[k] + atomicAdd(cur + k, 1)] = it;
}

// One thread per grid point (x fastest); the cells whose clouds reach point
// (i, j, k) are (i - dx, j - dy, k - dz), d in {0, 1}; the point is the upper
// corner (weight t) along a dimension where d = 1, the lower (1 - t) else.
__global__ void __launch_bounds__(TPB) k_cic_gather(int n, const int *__restrict__ start,
                                                    const CicItem *__restrict__ items, double *__restrict__ s0,
                                                    double *__restrict__ sx, double *__restrict__ sy,
                                                    double *__restrict__ sz, double *__restrict__ sm)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int cc = 0; cc < 8; ++cc) {
        const int dx = cc & 1, dy = (cc >> 1) & 1, dz = cc >> 2;
        const long c = lin(dx ? (i == 0 ? n - 1 : i - 1) : i, dy ? (j == 0 ? n - 1 : j - 1) : j,
                           dz ? (k == 0 ? n - 1 : k - 1) : k, n);
        const int b = start[c], e = start[c + 1];
        for (int s = b; s < e; ++s) {
            const CicItem it = items[s];
            const double w = (dx ? it.t[0] : 1.0 - it.t[0]) * (dy ? it.t[1] : 1.0 - it.t[1]) *
                             (dz ? it.t[2] : 1.0 - it.t[2]);
#pragma unroll
            for (int f = 0; f < 5; ++f) acc[f] += w * it.q[f];
        }
    }
    s0[p] = acc[0];
    sx[p] = acc[1];
    sy[p] = acc[2];
    sz[p] = acc[3];
    sm[p] = acc[4];
}

__global__ void k_fill_i32(int *__restrict__ x, long N, int v)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) x[p] = v;
}

// ----------------------------------------------------------------- builders

__global__ void k_shift_scale(double *__restrict__ out, const double *__restrict__ in, long N, double scale,
                              const double *__restrict__ mean)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) out[p] = scale * (in[p] - *mean);
}

// -1/4 d_j g^j
__global__ void k_div_quarter(double *__restrict__ out, const double *__restrict__ gx,
                              const double *__restrict__ gy, const double *__restrict__ gz, int n, double inv2h)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    out[p] = div_quarter_point(gx, gy, gz, i, j, k, n, inv2h);
}

struct A6Ptrs {
    double *c[6];
};

// A_ij and A_ijA^ij at every point
__global__ void __launch_bounds__(TPB) k_build_Aij(A6Ptrs A6, double *__restrict__ AA,
                                                   const double *__restrict__ Vx, const double *__restrict__ Vy,
                                                   const double *__restrict__ Vz, const double *__restrict__ U,
                                                   int n, double h)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    double A[6];
    AA[p] = aij_point(Vx, Vy, Vz, U, i, j, k, n, h, A);
    for (int c = 0; c < 6; ++c) A6.c[c][p] = A[c];
}

__global__ void k_ham_rhs(double *__restrict__ f, const double *__restrict__ s0, long N, double A)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < N) f[p] = A * (s0[p] - 1.0);
}

// CMC coefficient m2 and source f at every point
__global__ void k_build_cmc(double *__restrict__ m2, double *__restrict__ f, const double *__restrict__ psi,
                            const double *__restrict__ s0, const double *__restrict__ sm,
                            const double *__restrict__ AA, long N, double a, double om, double c)
{
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    cmc_point(psi[p], s0[p], sm[p], AA[p], a, om, c, m2[p], f[p]);
}

// sources of the three B^i equations at every point
__global__ void __launch_bounds__(TPB) k_shift_source(double *__restrict__ fBx, double *__restrict__ fBy,
                                                      double *__restrict__ fBz, const double *__restrict__ psi,
                                                      const double *__restrict__ xi, A6Ptrs A6, int n, double h,
                                                      double a, double c)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
    double out[3];
    shift_source_point(psi, xi, A6.c, i, j, k, n, h, a, c, out);
    fBx[p] = out[0];
    fBy[p] = out[1];
    fBz[p] = out[2];
}

// derived fields: 0 Phi = xi/chi, 1 alpha = 1 + Phi/(a^2c^2), 2 psi = a^(1/2) chi,
// 3 beta component = B + d_dir b (dir passed as which-3)
__global__ void k_derived(int which, double *__restrict__ out, const double *__restrict__ psi,
                          const double *__restrict__ xi, const double *__restrict__ Bc,
                          const double *__restrict__ b, int n, double h, double a, double c)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const double kap = 1.0 / (2.0 * a * a * c * c);
    if (which <= 2) {
        const double chi = 1.0 - kap * psi[p];
        if (which == 0) out[p] = xi[p] / chi;
        else if (which == 1) out[p] = 1.0 + (xi[p] / chi) / (a * a * c * c);
        else out[p] = sqrt(a) * chi;
    } else {
        const int dir = which - 3;
        const int i = (int)(p % n), j = (int)((p / n) % n), k = (int)(p / ((long)n * n));
        out[p] = Bc[p] + dcen(b, dir, i, j, k, n, 1.0 / (2.0 * h));
    }
}

inline unsigned blocks_for(long count) { return (unsigned)((count + TPB - 1) / TPB); }

} // namespace

void launch_cic_deposit(hipStream_t s, int n, double a, double c_tilde, const double *pos, const double *u,
                        double mass, long np, const double *psi, double *s0, double *sx, double *sy, double *sz,
                        double *sm)
{
    const double kap = 1.0 / (2.0 * a * a * c_tilde * c_tilde);
    if (np > 0)
        k_cic<<<blocks_for(np), TPB, 0, s>>>(n, a, c_tilde, kap, pos, u, mass, np, psi, s0, sx, sy, sz, sm);
}

size_t cic_sorted_bytes(long N, long cap)
{
    const long ntiles = (N + kScanTile - 1) / kScanTile;
    return sizeof(int) * (size_t)(2 * N + 1 + cap + ntiles) + sizeof(CicItem) * (size_t)cap + 8 * 256;
}

void launch_cic_sorted(hipStream_t s, int n, double a, double c_tilde, const double *pos, const double *u,
                       double mass, long np, const double *psi, void *scratch, double *s0, double *sx, double *sy,
                       double *sz, double *sm)
{
    const double kap = 1.0 / (2.0 * a * a * c_tilde * c_tilde);
    const long N = (long)n * n * n;
    const long ntiles = (N + kScanTile - 1) / kScanTile;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char *b = static_cast<char *>(scratch);
    CicItem *items = reinterpret_cast<CicItem *>(b);
    b += up(sizeof(CicItem) * (size_t)(np > 0 ? np : 1));
    int *start = reinterpret_cast<int *>(b); // N + 1
    b += up(sizeof(int) * (size_t)(N + 1));
    int *cnt = reinterpret_cast<int *>(b); // N, reused as the per-cell cursor
    b += up(sizeof(int) * (size_t)N);
    int *key = reinterpret_cast<int *>(b); // np
    b += up(sizeof(int) * (size_t)(np > 0 ? np : 1));
    int *tsum = reinterpret_cast<int *>(b); // ntiles
    k_fill_i32<<<blocks_for(N), TPB, 0, s>>>(cnt, N, 0);
    if (np > 0) k_cic_count<<<blocks_for(np), TPB, 0, s>>>(n, pos, np, key, cnt);
    k_scan_tiles<<<(unsigned)ntiles, TPB, 0, s>>>(cnt, N, start, tsum);
    k_scan_tile_sums<<<1, TPB, 0, s>>>(tsum, (int)ntiles, start + N);
    k_scan_add<<<blocks_for(N), TPB, 0, s>>>(start, N, tsum, cnt);
    if (np > 0)
        k_cic_place<<<blocks_for(np), TPB, 0, s>>>(n, a, c_tilde, kap, pos, u, mass, np, psi, key, start, cnt,
                                                    items);
    k_cic_gather<<<blocks_for(N), TPB, 0, s>>>(n, start, items, s0, sx, sy, sz, sm);
}

void launch_shift_scale(hipStream_t s, double *out, const double *in, long N, double scale, const double *mean)
{
    k_shift_scale<<<blocks_for(N), TPB, 0, s>>>(out, in, N, scale, mean);
}

void launch_div_quarter(hipStream_t s, double *out, const double *gx, const double *gy, const double *gz, int n,
                        double h)
{
    k_div_quarter<<<blocks_for((long)n * n * n), TPB, 0, s>>>(out, gx, gy, gz, n, 1.0 / (2.0 * h));
}

void launch_build_Aij(hipStream_t s, double *const A6[6], double *AA, const double *Vx, const double *Vy,
                      const double *Vz, const double *U, int n, double h)
{
    A6Ptrs P;
    for (int c = 0; c < 6; ++c) P.c[c] = A6[c];
    k_build_Aij<<<blocks_for((long)n * n * n), TPB, 0, s>>>(P, AA, Vx, Vy, Vz, U, n, h);
}

void launch_ham_rhs(hipStream_t s, double *f, const double *s0, long N, double A)
{
    k_ham_rhs<<<blocks_for(N), TPB, 0, s>>>(f, s0, N, A);
}

void launch_build_cmc(hipStream_t s, double *m2, double *f, const double *psi, const double *s0, const double *sm,
                      const double *AA, long N, double a, double om, double c_tilde)
{
    k_build_cmc<<<blocks_for(N), TPB, 0, s>>>(m2, f, psi, s0, sm, AA, N, a, om, c_tilde);
}

void launch_shift_source(hipStream_t s, double *fB[3], const double *psi, const double *xi, double *const A6[6],
                         int n, double h, double a, double c_tilde)
{
    A6Ptrs P;
    for (int c = 0; c < 6; ++c) P.c[c] = A6[c];
    k_shift_source<<<blocks_for((long)n * n * n), TPB, 0, s>>>(fB[0], fB[1], fB[2], psi, xi, P, n, h, a, c_tilde);
}

void launch_derived(hipStream_t s, int which, double *out, const double *psi, const double *xi, const double *Bc,
                    const double *b, int n, double h, double a, double c_tilde)
{
    k_derived<<<blocks_for((long)n * n * n), TPB, 0, s>>>(which, out, psi, xi, Bc, b, n, h, a, c_tilde);
}

} // namespace grmg
