// Vector-mode extraction (paper sec. 6.2): the shift beta^i -- likewise B^i
// and the momentum density s_i -- carries a scalar and a vector mode; the
// discrete curl removes the scalar one, and k^2 P_V(k) = P_curl(k) gives the
// vector mode's power.  Spectra are binned in |k| shells up to a quarter of
// the Nyquist wave number.
//
// Steps, all on the device:
//   1. curl and divergence by 3-point central differences, packed as two
//      complex fields z1 = curl_x + i curl_y, z2 = curl_z + i div (two real
//      transforms for the price of one complex transform each);
//   2. 3-D FFT of z1 and z2: one pass per axis, each workgroup transforming a
//      bundle of lines in LDS (radix-2 butterflies taken two stages at a time,
//      decimation in time from bit-reversed loads; y and z bundles take
//      consecutive x so every load is a row);
//   3. per mode of the cube |m_i| <= nbins: separate the four transforms with
//      F[a](m) = (Z(m) + conj Z(-m)) / 2, F[b](m) = (Z(m) - conj Z(-m)) / (2i),
//      form the curl and divergence power and their ratio to |k_eff|^2, and
//      add them to the mode's shell in a fixed order (per-block partial sums
//      over 256-mode chunks, then a fixed-order sum over blocks).
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <new>
#include <string>

#include <hip/hip_runtime.h>

#include "gr.h"

namespace {

constexpr int TPB = 256;
constexpr int kFftLds = 4096;  // complex doubles of line data per workgroup (64 KiB)
constexpr int kMaxN = 1024;    // twiddle table in LDS: n / 2 entries
constexpr int kRows = 6;       // k, count, P_curl, P_div, P_vector, P_scalar
constexpr int kTargetBlocks = 512;

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// tw[j] = exp(-2 pi i j / n), j < n / 2
__global__ void k_twiddles(double2 *__restrict__ tw, int n)
{
    const int j = blockIdx.x * TPB + threadIdx.x;
    if (j >= n / 2) return;
    double s, c;
    sincospi(-2.0 * j / n, &s, &c);
    tw[j] = double2{c, s};
}

// z1 = curl_x + i curl_y, z2 = curl_z + i div at every cell
__global__ void __launch_bounds__(TPB) k_curl_div(const double *__restrict__ vx, const double *__restrict__ vy,
                                                  const double *__restrict__ vz, int n, double2 *__restrict__ z1,
                                                  double2 *__restrict__ z2)
{
    const long N = (long)n * n * n;
    const long p = (long)blockIdx.x * TPB + threadIdx.x;
    if (p >= N) return;
    const int x = (int)(p % n), y = (int)((p / n) % n), z = (int)(p / ((long)n * n));
    const long row = p - x, plane = (long)n * n;
    const long xp = row + wrapi(x + 1, n), xm = row + wrapi(x - 1, n);
    const long yp = p + (long)(wrapi(y + 1, n) - y) * n, ym = p + (long)(wrapi(y - 1, n) - y) * n;
    const long zp = p + (long)(wrapi(z + 1, n) - z) * plane, zm = p + (long)(wrapi(z - 1, n) - z) * plane;
    const double f = 0.5 * n;
    const double dyvz = (vz[yp] - vz[ym]) * f, dzvy = (vy[zp] - vy[zm]) * f;
    const double dzvx = (vx[zp] - vx[zm]) * f, dxvz = (vz[xp] - vz[xm]) * f;
    const double dxvy = (vy[xp] - vy[xm]) * f, dyvx = (vx[yp] - vx[ym]) * f;
    const double dxvx = (vx[xp] - vx[xm]) * f, dyvy = (vy[yp] - vy[ym]) * f, dzvz = (vz[zp] - vz[zm]) * f;
    z1[p] = double2{dyvz - dzvy, dzvx - dxvz};
    z2[p] = double2{dxvy - dyvx, dxvx + dyvy + dzvz};
}

// The same for n >= 64 by z-marching columns: a workgroup takes a 64 x 4
// tile of (x, y) columns over kCdz planes, each thread keeping its column's
// values at z - 1, z and z + 1 in registers (x and y neighbours are the
// adjacent columns' loads, cache hits when the neighbouring tile ran on the
// same XCD); identical arithmetic per cell.
constexpr int kCdx = 64, kCdy = 4, kCdz = 16;
__global__ void __launch_bounds__(TPB) k_curl_div_march(const double *__restrict__ vx, const double *__restrict__ vy,
                                                        const double *__restrict__ vz, int n,
                                                        double2 *__restrict__ z1, double2 *__restrict__ z2)
{
    const int ntx = n / kCdx, nty = n / kCdy;
    // XCD-contiguous order (the grid is a multiple of 8): each XCD takes one run
    // of consecutive tiles, so the y-neighbour rows of a tile sit in its L2
    const int G = gridDim.x, v = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
    const int bx = v % ntx, by = (v / ntx) % nty, bz = v / (ntx * nty);
    const int x = bx * kCdx + (threadIdx.x & (kCdx - 1)), y = by * kCdy + (threadIdx.x >> 6), z0 = bz * kCdz;
    const int xp = wrapi(x + 1, n), xm = wrapi(x - 1, n), yp = wrapi(y + 1, n), ym = wrapi(y - 1, n);
    const double f = 0.5 * n;
    auto at = [&](int xx, int yy, int zz) { return ((long)zz * n + yy) * n + xx; };
    const long pm = at(x, y, wrapi(z0 - 1, n)), pc = at(x, y, z0);
    double px = vx[pm], py = vy[pm], pz = vz[pm];
    double cx = vx[pc], cy = vy[pc], cz = vz[pc];
    for (int z = z0; z < z0 + kCdz; ++z) {
        const long p = at(x, y, z), pn = at(x, y, wrapi(z + 1, n));
        const double nx = vx[pn], ny = vy[pn], nz = vz[pn];
        const long xP = p - x + xp, xM = p - x + xm, yP = p + (long)(yp - y) * n, yM = p + (long)(ym - y) * n;
        const double dyvz = (vz[yP] - vz[yM]) * f, dzvy = (ny - py) * f;
        const double dzvx = (nx - px) * f, dxvz = (vz[xP] - vz[xM]) * f;
        const double dxvy = (vy[xP] - vy[xM]) * f, dyvx = (vx[yP] - vx[yM]) * f;
        const double dxvx = (vx[xP] - vx[xM]) * f, dyvy = (vy[yP] - vy[yM]) * f, dzvz = (nz - pz) * f;
        z1[p] = double2{dyvz - dzvy, dzvx - dxvz};
        z2[p] = double2{dxvy - dyvx, dxvx + dyvy + dzvz};
        px = cx;
        py = cy;
        pz = cz;
        cx = nx;
        cy = ny;
        cz = nz;
    }
}

// In-place forward transform of every line along AXIS (0 = x, 1 = y, 2 = z)
// of an n^3 complex array; a workgroup takes lb lines (lb * n <= kFftLds).
template <int AXIS>
__global__ void __launch_bounds__(TPB) k_fft_lines(double2 *__restrict__ data, int n, int logn, int loglb,
                                                   const double2 *__restrict__ tw)
{
    __shared__ double2 s[kFftLds];
    __shared__ double2 stw[kMaxN / 2];
    const int tid = threadIdx.x;
    const int lb = 1 << loglb, half = n >> 1, tot = lb << logn;
    for (int j = tid; j < half; j += TPB) stw[j] = tw[j];
    const long n2 = (long)n * n;
    long base, lstride, jstride;
    if (AXIS == 0) {
        base = (long)blockIdx.x * tot;
        lstride = n;
        jstride = 1;
    } else {
        const int nxb = n >> loglb;
        const long x0 = (long)(blockIdx.x % nxb) << loglb, other = blockIdx.x / nxb;
        base = AXIS == 1 ? other * n2 + x0 : other * n + x0;
        lstride = 1;
        jstride = AXIS == 1 ? n : n2;
    }
    const int shift = 32 - logn;
    for (int idx = tid; idx < tot; idx += TPB) {
        const int l = AXIS == 0 ? idx >> logn : idx & (lb - 1);
        const int j = AXIS == 0 ? idx & (n - 1) : idx >> loglb;
        s[(l << logn) + (int)(__brev((unsigned)j) >> shift)] = data[base + l * lstride + j * jstride];
    }
    __syncthreads();
    // radix-2 stages in pairs (one LDS round trip and barrier per pair): the
    // same butterflies and twiddles as stage after stage; an odd first stage alone
    int ls = 0;
    if (logn & 1) {
        for (int bi = tid; bi < (tot >> 1); bi += TPB) {
            const int l = bi >> (logn - 1), t = bi & (half - 1);
            const int i0 = (l << logn) + (t << 1), i1 = i0 + 1;
            const double2 a = s[i0], c = s[i1]; // twiddle 1
            s[i0] = double2{a.x + c.x, a.y + c.y};
            s[i1] = double2{a.x - c.x, a.y - c.y};
        }
        __syncthreads();
        ls = 1;
    }
    for (; ls < logn; ls += 2) {
        const int hs = 1 << ls, t1 = logn - 1 - ls, t2 = logn - 2 - ls;
        for (int gi = tid; gi < (tot >> 2); gi += TPB) {
            const int l = gi >> (logn - 2), t = gi & ((n >> 2) - 1);
            const int k = t & (hs - 1), grp = t >> ls;
            const int i0 = (l << logn) + (grp << (ls + 2)) + k;
            const double2 a0 = s[i0], a1 = s[i0 + hs], a2 = s[i0 + 2 * hs], a3 = s[i0 + 3 * hs];
            const double2 w1 = stw[k << t1];
            const double b1x = a1.x * w1.x - a1.y * w1.y, b1y = a1.x * w1.y + a1.y * w1.x;
            const double b3x = a3.x * w1.x - a3.y * w1.y, b3y = a3.x * w1.y + a3.y * w1.x;
            const double2 c0{a0.x + b1x, a0.y + b1y}, c1{a0.x - b1x, a0.y - b1y};
            const double2 c2{a2.x + b3x, a2.y + b3y}, c3{a2.x - b3x, a2.y - b3y};
            const double2 w2 = stw[k << t2], w3 = stw[(k + hs) << t2];
            const double d2x = c2.x * w2.x - c2.y * w2.y, d2y = c2.x * w2.y + c2.y * w2.x;
            const double d3x = c3.x * w3.x - c3.y * w3.y, d3y = c3.x * w3.y + c3.y * w3.x;
            s[i0] = double2{c0.x + d2x, c0.y + d2y};
            s[i0 + 2 * hs] = double2{c0.x - d2x, c0.y - d2y};
            s[i0 + hs] = double2{c1.x + d3x, c1.y + d3y};
            s[i0 + 3 * hs] = double2{c1.x - d3x, c1.y - d3y};
        }
        __syncthreads();
    }
    for (int idx = tid; idx < tot; idx += TPB) {
        const int l = AXIS == 0 ? idx >> logn : idx & (lb - 1);
        const int j = AXIS == 0 ? idx & (n - 1) : idx >> loglb;
        data[base + l * lstride + j * jstride] = s[(l << logn) + j];
    }
}

// Shell sums over the modes m in [-R, R]^3 (R = nbins), 256 modes per chunk,
// `chunks` chunks per block; thread t < nbins adds shell t's entries of each
// chunk in mode order.  part[block][row][nbins].
__global__ void __launch_bounds__(TPB) k_bin_modes(const double2 *__restrict__ z1, const double2 *__restrict__ z2,
                                                   int n, int nbins, long nmodes, int chunks,
                                                   double *__restrict__ part)
{
    __shared__ int sbin[TPB];
    __shared__ double sval[kRows][TPB];
    const int tid = threadIdx.x;
    const int R = nbins, S = 2 * R + 1;
    const double N = (double)n * n * n, invN2 = 1.0 / (N * N), twopi = 6.283185307179586476925286766559;
    double acc[kRows] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < chunks; ++c) {
        const long q = ((long)blockIdx.x * chunks + c) * TPB + tid;
        int bin = -1;
        double v[kRows] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (q < nmodes) {
            const int mx = (int)(q % S) - R, my = (int)((q / S) % S) - R, mz = (int)(q / ((long)S * S)) - R;
            const double mag = sqrt((double)(mx * mx + my * my + mz * mz));
            bin = (int)floor(mag + 0.5) - 1;
            if (bin >= 0 && bin < nbins) {
                const long ip = ((long)wrapi(mz, n) * n + wrapi(my, n)) * n + wrapi(mx, n);
                const long im = ((long)wrapi(-mz, n) * n + wrapi(-my, n)) * n + wrapi(-mx, n);
                const double2 ap = z1[ip], am = z1[im], bp = z2[ip], bm = z2[im];
                // F[curl_x] = (ap + conj am) / 2, F[curl_y] = (ap - conj am) / (2i), likewise curl_z, div from z2
                const double fxr = 0.5 * (ap.x + am.x), fxi = 0.5 * (ap.y - am.y);
                const double fyr = 0.5 * (ap.y + am.y), fyi = -0.5 * (ap.x - am.x);
                const double fzr = 0.5 * (bp.x + bm.x), fzi = 0.5 * (bp.y - bm.y);
                const double fdr = 0.5 * (bp.y + bm.y), fdi = -0.5 * (bp.x - bm.x);
                const double pc = ((fxr * fxr + fxi * fxi) + (fyr * fyr + fyi * fyi) + (fzr * fzr + fzi * fzi)) * invN2;
                const double pd = (fdr * fdr + fdi * fdi) * invN2;
                double sx, sy, sz, cc;
                sincospi(2.0 * mx / n, &sx, &cc);
                sincospi(2.0 * my / n, &sy, &cc);
                sincospi(2.0 * mz / n, &sz, &cc);
                const double keff2 = (n * sx) * (n * sx) + (n * sy) * (n * sy) + (n * sz) * (n * sz);
                v[0] = twopi * mag;
                v[1] = 1.0;
                v[2] = pc;
                v[3] = pd;
                v[4] = pc / keff2;
                v[5] = pd / keff2;
            } else {
                bin = -1;
            }
        }
        sbin[tid] = bin;
#pragma unroll
        for (int r = 0; r < kRows; ++r) sval[r][tid] = v[r];
        __syncthreads();
        if (tid < nbins)
            for (int e = 0; e < TPB; ++e)
                if (sbin[e] == tid)
#pragma unroll
                    for (int r = 0; r < kRows; ++r) acc[r] += sval[r][e];
        __syncthreads();
    }
    if (tid < nbins)
#pragma unroll
        for (int r = 0; r < kRows; ++r) part[((long)blockIdx.x * kRows + r) * nbins + tid] = acc[r];
}

// out[row][bin] = sum over blocks, in block order
__global__ void k_bin_reduce(const double *__restrict__ part, int nblk, int cells, double *__restrict__ out)
{
    const int q = blockIdx.x * TPB + threadIdx.x;
    if (q >= cells) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(long)b * cells + q];
    out[q] = s;
}

thread_local std::string s_err;
int sfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int sfail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s_err = buf;
    return code;
}
#define SHIP(expr)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return sfail(GR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)
#define SLAUNCH() SHIP(hipGetLastError())

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

} // namespace

struct gr_spectra_s {
    int n = 0, logn = 0, nbins = 0;
    long nmodes = 0;
    int chunks = 1, nblk = 0;
    size_t off_z1 = 0, off_z2 = 0, off_tw = 0, off_part = 0, off_out = 0, bytes = 0;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
};

namespace {

int fft3(gr_spectra S, double2 *d)
{
    const int n = S->n, logn = S->logn;
    const int lb = n < kFftLds / n ? n : kFftLds / n, loglb = ilog2(lb);
    const unsigned grid = (unsigned)((long)n * n / lb);
    const double2 *tw = reinterpret_cast<const double2 *>(S->ws + S->off_tw);
    k_fft_lines<0><<<grid, TPB, 0, S->stream>>>(d, n, logn, loglb, tw);
    k_fft_lines<1><<<grid, TPB, 0, S->stream>>>(d, n, logn, loglb, tw);
    k_fft_lines<2><<<grid, TPB, 0, S->stream>>>(d, n, logn, loglb, tw);
    SLAUNCH();
    return GR_OK;
}

} // namespace

extern "C" {

const char *gr_spectra_last_error(void) { return s_err.c_str(); }

int gr_create_spectra(int n, int nbins, gr_spectra *out)
{
    if (!out) return sfail(GR_EINVAL, "null argument");
    *out = nullptr;
    if (n < 8 || n > kMaxN || (n & (n - 1))) return sfail(GR_EINVAL, "n = %d must be a power of two in [8, %d]", n, kMaxN);
    if (nbins < 1 || nbins > n / 4) return sfail(GR_EINVAL, "nbins = %d must be in [1, n/4 = %d]", nbins, n / 4);
    gr_spectra S = new (std::nothrow) gr_spectra_s;
    if (!S) return sfail(GR_EDEVICE, "out of host memory");
    S->n = n;
    S->logn = ilog2(n);
    S->nbins = nbins;
    const long side = 2L * nbins + 1;
    S->nmodes = side * side * side;
    const long chunks_total = (S->nmodes + TPB - 1) / TPB;
    S->chunks = (int)((chunks_total + kTargetBlocks - 1) / kTargetBlocks);
    S->nblk = (int)((chunks_total + S->chunks - 1) / S->chunks);
    const size_t N = (size_t)n * n * n;
    size_t off = 0;
    S->off_z1 = off;
    off += al256(N * sizeof(double2));
    S->off_z2 = off;
    off += al256(N * sizeof(double2));
    S->off_tw = off;
    off += al256((size_t)(n / 2) * sizeof(double2));
    S->off_part = off;
    off += al256((size_t)S->nblk * kRows * nbins * sizeof(double));
    S->off_out = off;
    off += al256((size_t)kRows * nbins * sizeof(double));
    S->bytes = off;
    *out = S;
    return GR_OK;
}

int gr_spectra_workspace_bytes(gr_spectra S, size_t *bytes)
{
    if (!S || !bytes) return sfail(GR_EINVAL, "null argument");
    *bytes = S->bytes;
    return GR_OK;
}

int gr_spectra_bind(gr_spectra S, void *d_ws, size_t bytes, void *stream)
{
    if (!S || !d_ws) return sfail(GR_EINVAL, "null argument");
    if (bytes < S->bytes) return sfail(GR_EINVAL, "workspace %zu bytes < required %zu", bytes, S->bytes);
    if (reinterpret_cast<uintptr_t>(d_ws) % 256) return sfail(GR_EINVAL, "workspace not 256-byte aligned");
    S->ws = reinterpret_cast<char *>(d_ws);
    S->stream = reinterpret_cast<hipStream_t>(stream);
    k_twiddles<<<(unsigned)((S->n / 2 + TPB - 1) / TPB), TPB, 0, S->stream>>>(
        reinterpret_cast<double2 *>(S->ws + S->off_tw), S->n);
    SLAUNCH();
    S->bound = true;
    return GR_OK;
}

int gr_spectra_fft(gr_spectra S, double *d_data)
{
    if (!S || !d_data) return sfail(GR_EINVAL, "null argument");
    if (!S->bound) return sfail(GR_ESTATE, "spectra handle not bound");
    if (reinterpret_cast<uintptr_t>(d_data) % 16) return sfail(GR_EINVAL, "data not 16-byte aligned");
    return fft3(S, reinterpret_cast<double2 *>(d_data));
}

int gr_vector_spectra(gr_spectra S, const double *d_vx, const double *d_vy, const double *d_vz, double *h_out)
{
    if (!S || !d_vx || !d_vy || !d_vz || !h_out) return sfail(GR_EINVAL, "null argument");
    if (!S->bound) return sfail(GR_ESTATE, "spectra handle not bound");
    const int n = S->n, nb = S->nbins;
    const long N = (long)n * n * n;
    double2 *z1 = reinterpret_cast<double2 *>(S->ws + S->off_z1);
    double2 *z2 = reinterpret_cast<double2 *>(S->ws + S->off_z2);
    double *part = reinterpret_cast<double *>(S->ws + S->off_part);
    double *out = reinterpret_cast<double *>(S->ws + S->off_out);
    if (n >= kCdx)
        k_curl_div_march<<<(unsigned)((n / kCdx) * (n / kCdy) * (n / kCdz)), TPB, 0, S->stream>>>(d_vx, d_vy, d_vz, n,
                                                                                                 z1, z2);
    else
        k_curl_div<<<(unsigned)((N + TPB - 1) / TPB), TPB, 0, S->stream>>>(d_vx, d_vy, d_vz, n, z1, z2);
    SLAUNCH();
    int rc = fft3(S, z1);
    if (rc != GR_OK) return rc;
    rc = fft3(S, z2);
    if (rc != GR_OK) return rc;
    k_bin_modes<<<(unsigned)S->nblk, TPB, 0, S->stream>>>(z1, z2, n, nb, S->nmodes, S->chunks, part);
    const int cells = kRows * nb;
    k_bin_reduce<<<(unsigned)((cells + TPB - 1) / TPB), TPB, 0, S->stream>>>(part, S->nblk, cells, out);
    SLAUNCH();
    SHIP(hipMemcpyAsync(h_out, out, (size_t)cells * sizeof(double), hipMemcpyDeviceToHost, S->stream));
    SHIP(hipStreamSynchronize(S->stream));
    // sums -> means over each shell's modes
    for (int b = 0; b < nb; ++b) {
        const double c = h_out[nb + b];
        if (c > 0)
            for (int r = 0; r < kRows; ++r)
                if (r != 1) h_out[r * nb + b] /= c;
    }
    return GR_OK;
}

int gr_destroy_spectra(gr_spectra S)
{
    delete S;
    return GR_OK;
}

} // extern "C"
