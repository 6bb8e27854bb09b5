// Batched solve of many independent periodic boxes of uneven size, and of
// Dirichlet refinement patches whose boundary values come from a box of the
// same batch (patch_ops.h).
//
// Every phase of the multigrid cycle is one launch over all boxes: a prefix
// table maps each block to its box, and each box's slice of the launch works
// on that box's own arrays.  Stopping is decided per box on the device (a
// converged box's blocks return at once), so the host only reads one word per
// cycle ("is any box still active?"), and the whole per-cycle sequence is
// captured once per field in a hipGraph and replayed.  The arithmetic of
// every step is the single-grid arithmetic (shared device functions), so each
// box gets exactly the cycle of the single-grid solver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sources_ops.h"
#include "patch_ops.h"
#include "fused_sweep.h"
#include "coarse_cycle.h"
#include "march.h"

using namespace grmg;
using namespace grmg::detail;

namespace {

constexpr int TPB = 256;
constexpr int kSumPPT = 8; // points per thread of the batch sums and mean subtraction
constexpr int CTPB = 1024;
constexpr int kMaxBoxes = 4096;

// device-side description of one box
struct BoxLev {
    int n;
    double h;
    double *phi, *phi0, *f, *coef, *tmp; // phi of level 0 is the current field array
    double *ptmp; // patch levels swept fused: padded scratch iterate (its faces hold the boundary values too)
    // mixed precision (periodic boxes): FP32 correction e, its source b, the
    // frozen linearisation a (chi) and c, scratch
    float *e, *b32, *a32, *c32, *t32;
};
struct BoxDev {
    int nlev;
    int centry; // first level handled by the single-workgroup coarse cycle
    int qentry; // first level run by the device task queue (== centry: only the coarse cycle)
    int centry32; // first level of the FP32 correction cycle handled by the single-workgroup kernel
    int patch;  // 1: Dirichlet patch (padded iterate arrays), 0: periodic box
    int parent; // patch: index of the item (periodic box or earlier patch) its boundary values come from
    int depth;  // 0: periodic box; patch: its parent's depth + 1
    double origin[3]; // patch: lower corner in the parent's frame (box units)
    double *field[10];
    double *src[5];
    double *A6[6];
    double *AA;
    double *fB[3];
    BoxLev lev[kMaxLevels];
};

// per-box scalars (device)
// B_ZERO stays 0; B_PREV, B_STALL, B_FB: mixed precision's previous relative
// residual, count of stalled refinement steps in a row, and fallback flag
enum BoxScal { B_FBAR, B_FSHIFT, B_FMEAN, B_MEAN, B_RN, B_FN, B_REL, B_TMP, B_ZERO, B_PREV, B_STALL, B_FB, B_NSCAL };

struct BatchDev {
    const BoxDev *box;
    double *scal;   // [nbox][B_NSCAL]
    int *active;    // [nbox]
    int *cycles;    // [nbox][10]
    int *status;    // [nbox]
    unsigned long long *t_done; // [nbox][10] device clock at convergence
    unsigned long long *t_start; // [20]: periodic boxes' fields, then patches' fields
    int *any_active;
    double *partials;
    int nbox;
    int march; // the stopping norms and residual + restriction use the plane-marching form where it applies
};

__device__ __forceinline__ int find_box(const int *__restrict__ start, int nbox, int blk)
{
    int lo = 0, hi = nbox;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// decode item t of an nx x ny x nz domain (x fastest)
__device__ __forceinline__ void decode3(int t, int nx, int ny, int &x, int &y, int &z)
{
    x = t % nx;
    const int r = t / nx;
    y = r % ny;
    z = r / ny;
}

#define BOX_PROLOGUE(tab)                                                                             \
    const int b = find_box(tab, D.nbox, blockIdx.x);                                                 \
    const BoxDev &X = D.box[b];                                                                       \
    const int t = (blockIdx.x - tab[b]) * TPB + threadIdx.x;

// ----------------------------------------------------------- multigrid phases

template <int KIND>
__global__ void __launch_bounds__(TPB) kb_colour(BatchDev D, const int *__restrict__ tab, int d, int fid, int colour,
                                                 OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &L = X.lev[d];
    const int n = L.n, half = n >> 1;
    if (t >= n * n * half) return;
    int x2, y, z;
    decode3(t, half, n, x2, y, z);
    const int i = 2 * x2 + ((y + z + colour) & 1);
    double *phi = d == 0 ? X.field[fid] : L.phi;
    const long p = lin(i, y, z, n);
    const double Fb = d == 0 ? D.scal[b * B_NSCAL + B_FBAR] : 0.0;
    const double fs = d == 0 ? D.scal[b * B_NSCAL + B_FSHIFT] : 0.0;
    const double ph = phi[p];
    double J;
    const double Lv = op_point<KIND, double>(ph, nb_sum(phi, i, y, z, n), 1.0 / (L.h * L.h), load_c1<KIND>(L.coef, p),
                                             0.0, oc, Fb, J);
    phi[p] = ph - (Lv - (L.f[p] - fs)) / J;
}

// Fused red-black sweeps (rb_fused_tile) of the boxes whose level d takes
// TX x TY tiles (32x16 or 64x16): one workgroup per tile x 16-plane chunk, the
// box from the block prefix table.  Out of place: even sweeps phi -> tmp, odd
// tmp -> phi.
constexpr int kFZ = 16; // z-chunk of the batched fused sweep

template <int KIND, int TX, int TY>
__global__ void __launch_bounds__((TX / 2) * TY) kb_fused(BatchDev D, const int *__restrict__ tab, int d, int fid,
                                                          int sweep, OpConst oc)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const BoxLev &L = X.lev[d];
    const int n = L.n, lb = blockIdx.x - tab[b];
    const int nz = n / kFZ, tiles_y = n / TY;
    const int zchunk = lb % nz, t2 = lb / nz;
    double *phi = d == 0 ? X.field[fid] : L.phi;
    const double *in = (sweep & 1) ? L.tmp : phi;
    double *out = (sweep & 1) ? phi : L.tmp;
    const double Fb = d == 0 ? D.scal[b * B_NSCAL + B_FBAR] : 0.0;
    const double fs = d == 0 ? D.scal[b * B_NSCAL + B_FSHIFT] : 0.0;
    constexpr int PF = KIND == GR_KIND_POISSON ? 2 : 1;
    rb_fused_tile<KIND, double, TX, TY, PF>(in, out, L.f, L.coef, nullptr, n, kFZ, 1.0 / (L.h * L.h), oc, Fb, fs,
                                            (t2 / tiles_y) * TX, (t2 % tiles_y) * TY, zchunk * kFZ);
}


template <int KIND>
__global__ void __launch_bounds__(TPB) kb_coarse_rhs(BatchDev D, const int *__restrict__ tab, int d, OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &C = X.lev[d + 1];
    const int m = C.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    double Jd;
    const double Lv = op_point<KIND, double>(C.phi[t], nb_sum(C.phi, I, J, K, m), 1.0 / (C.h * C.h),
                                             load_c1<KIND>(C.coef, t), 0.0, oc, 0.0, Jd);
    C.f[t] = Lv - C.tmp[t];
}


// coarse correction e = phi^H - R phi into level d+1's tmp (free once the
// coarse source is built), one thread per coarse cell
__global__ void __launch_bounds__(TPB) kb_coarse_diff(BatchDev D, const int *__restrict__ tab, int d)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &C = X.lev[d + 1];
    const int m = C.n;
    if (t >= m * m * m) return;
    C.tmp[t] = C.phi[t] - C.phi0[t];
}

// phi += P e from level d+1's tmp: one thread per coarse cell writes its 8
// children (x-pairs as 16-byte read-modify-writes); same weights and order
// as the single-point form
__global__ void __launch_bounds__(TPB) kb_prolong_cell(BatchDev D, const int *__restrict__ tab, int d, int fid)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &L = X.lev[d], &C = X.lev[d + 1];
    const int n = L.n, m = C.n;
    if (t >= m * m * m) return;
    int x, y, z;
    decode3(t, m, m, x, y, z);
    double *phi = d == 0 ? X.field[fid] : L.phi;
    double e[3][3][3];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                e[dz + 1][dy + 1][dx + 1] = C.tmp[lin(wrapi(x + dx, m), wrapi(y + dy, m), wrapi(z + dz, m), m)];
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy) {
            double v[2];
            for (int cx = 0; cx < 2; ++cx) {
                const int sx = cx ? 1 : -1, sy = cy ? 1 : -1, sz = cz ? 1 : -1;
                double a = 0.0;
                for (int c = 0; c < 8; ++c) {
                    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                    const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
                    a += w * e[1 + oz * sz][1 + oy * sy][1 + ox * sx];
                }
                v[cx] = a;
            }
            double2 *dst = reinterpret_cast<double2 *>(phi + lin(2 * x, 2 * y + cy, 2 * z + cz, n));
            double2 old = *dst;
            old.x += v[0];
            old.y += v[1];
            *dst = old;
        }
}

// coefficient restriction level d -> d+1 (once per solve of an equation)
__global__ void __launch_bounds__(TPB) kb_restrict_coef(BatchDev D, const int *__restrict__ tab, int d)
{
    BOX_PROLOGUE(tab)
    const BoxLev &L = X.lev[d], &C = X.lev[d + 1];
    const int m = C.n, n = L.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += L.coef[lin(2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2), n)];
    C.coef[t] = s / 8.0;
}

// the rest of the V-cycle of each active box from its entry level, one workgroup per box
template <int KIND>
__global__ void __launch_bounds__(CTPB) kb_coarse_vcycle(BatchDev D, int fid, int nu1, int nu2, OpConst oc);

// ------------------------------------------------------------- reductions

// per-block partial sums (fixed order) of the fine level of each box
template <int NC>
__device__ __forceinline__ void block_store(double (&v)[NC], double *__restrict__ partials, int total_blocks)
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
            partials[c * total_blocks + blockIdx.x] = s;
        }
    }
}

// what: 0 sum(phi), 1 sum F (Hamiltonian), 2 sum(m2 phi), 3 sum(f), 4..6 sum(s_x..s_z), 7 sum(e) (FP32 correction)
// PPT points per thread (strided by the block size, so each pass is coalesced);
// the table gives each box ceil(n^3 / (PPT TPB)) blocks
template <int PPT>
__global__ void __launch_bounds__(TPB) kb_sum(BatchDev D, const int *__restrict__ tab, int fid, int what, OpConst oc,
                                              int active_only)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    const BoxDev &X = D.box[b];
    const int total = tab[D.nbox];
    double v[1] = {0.0};
    const BoxLev &L = X.lev[0];
    const int N = L.n * L.n * L.n;
    if (!active_only || D.active[b]) {
        const int t0 = (blockIdx.x - tab[b]) * TPB * PPT + threadIdx.x;
        // every load of the thread is issued before the first is used
        double x[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int t = t0 + q * TPB;
            const bool in = t < N;
            const int tc = in ? t : 0;
            double val;
            if (what == 0) val = X.field[fid][tc];
            else if (what == 1) {
                const double chi = 1.0 - oc.kappa * X.field[fid][tc];
                const double chi2 = chi * chi;
                const double chi6 = chi2 * chi2 * chi2;
                const double chim7 = 1.0 / (chi6 * chi);
                val = (L.f[tc] - oc.A * (chi6 - 1.0)) / chi + 0.25 * L.coef[tc] * chim7;
            } else if (what == 2) val = L.coef[tc] * X.field[fid][tc];
            else if (what == 3) val = L.f[tc];
            else if (what == 7) val = (double)X.lev[0].e[tc];
            else val = X.src[what - 3][tc];
            x[q] = in ? val : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q) v[0] += x[q];
    }
    block_store<1>(v, D.partials, total);
}


// Plane-marching forms (march_tile, 16-plane chunks) for boxes whose level
// takes 32 x 8 tiles, the one-thread-per-point forms for the others, in one
// launch: the table gives each box its blocks for whichever form it takes.
// z-chunk of the plane-marching forms: 32 planes for the large boxes, 16 for the others
__host__ __device__ inline int mz_chunk(int n) { return n >= 96 ? 32 : 16; }

__host__ __device__ inline bool marchable(int n) { return n >= 64 && n % 32 == 0; }
__host__ __device__ inline long march_blocks(int n) { return (long)(n / MTX) * (n / MTY) * (n / mz_chunk(n)); }

template <int KIND>
__global__ void __launch_bounds__(TPB) kb_norms_m(BatchDev D, const int *__restrict__ tab, int fid, OpConst oc)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    const BoxDev &X = D.box[b];
    const int total = tab[D.nbox];
    const int lb = blockIdx.x - tab[b];
    const BoxLev &L = X.lev[0];
    const int n = L.n;
    const double Fb = D.scal[b * B_NSCAL + B_FBAR], fs = D.scal[b * B_NSCAL + B_FSHIFT];
    double v[2] = {0.0, 0.0};
    if (D.active[b]) {
        const double *phi = X.field[fid];
        if (D.march && marchable(n)) { // the block table gives march_blocks(n) blocks
            const int mz = mz_chunk(n), nzc = n / mz, tiles_y = n / MTY, tile = lb / nzc, zchunk = lb % nzc;
            march_tile<M_NORMS, KIND, double>(phi, L.f, L.coef, nullptr, n, mz, 1.0 / (L.h * L.h), oc, Fb, fs,
                                              (tile / tiles_y) * MTX, (tile % tiles_y) * MTY, zchunk * mz, nullptr,
                                              nullptr, nullptr, nullptr, nullptr, nullptr, v);
        } else {
            const int t = lb * TPB + threadIdx.x;
            if (t < n * n * n) {
                int x, y, z;
                decode3(t, n, n, x, y, z);
                double Jd;
                const double Lv = op_point<KIND, double>(phi[t], nb_sum(phi, x, y, z, n), 1.0 / (L.h * L.h),
                                                         load_c1<KIND>(L.coef, t), 0.0, oc, Fb, Jd);
                const double fe = L.f[t] - fs;
                const double e = Lv - fe;
                v[0] = e * e;
                v[1] = fe * fe;
            }
        }
    }
    block_store<2>(v, D.partials, total);
}

template <int KIND>
__global__ void __launch_bounds__(TPB) kb_rr_m(BatchDev D, const int *__restrict__ tab, int d, int fid, OpConst oc)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const int lb = blockIdx.x - tab[b];
    const BoxLev &L = X.lev[d], &C = X.lev[d + 1];
    const int n = L.n;
    const double *phi = d == 0 ? X.field[fid] : L.phi;
    const double Fb = d == 0 ? D.scal[b * B_NSCAL + B_FBAR] : 0.0;
    const double fs = d == 0 ? D.scal[b * B_NSCAL + B_FSHIFT] : 0.0;
    if (D.march && marchable(n)) { // the block table gives march_blocks(n) blocks
        const int mz = mz_chunk(n), nzc = n / mz, tiles_y = n / MTY, tile = lb / nzc, zchunk = lb % nzc;
        double v[2];
        march_tile<M_RESTRICT, KIND, double>(phi, L.f, L.coef, nullptr, n, mz, 1.0 / (L.h * L.h), oc, Fb, fs,
                                             (tile / tiles_y) * MTX, (tile % tiles_y) * MTY, zchunk * mz, C.phi,
                                             C.phi0, C.tmp, nullptr, nullptr, nullptr, v);
        return;
    }
    const int m = C.n, t = lb * TPB + threadIdx.x;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    const double inv_h2 = 1.0 / (L.h * L.h);
    double sr = 0.0, sp = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
        const long p = lin(i, j, k, n);
        const double ph = phi[p];
        double Jd;
        const double Lv = op_point<KIND, double>(ph, nb_sum(phi, i, j, k, n), inv_h2, load_c1<KIND>(L.coef, p), 0.0,
                                                 oc, Fb, Jd);
        sr += Lv - (L.f[p] - fs);
        sp += ph;
    }
    const double rp = sp / 8.0;
    C.phi[t] = rp;
    C.phi0[t] = rp;
    C.tmp[t] = sr / 8.0;
}

// per item b0 + blockIdx.x: slot[c] = add_slot + 1/N * sum of its block partials of component c
__global__ void __launch_bounds__(TPB) kb_finalize(BatchDev D, const int *__restrict__ tab, int ncomp, int slot,
                                                   int add_slot, int active_only, int b0)
{
    const int b = b0 + blockIdx.x;
    if (active_only && !D.active[b]) return;
    const int total = tab[D.nbox];
    const int n = D.box[b].lev[0].n;
    const double invN = 1.0 / ((double)n * n * n);
    __shared__ double sh[TPB];
    for (int c = 0; c < ncomp; ++c) {
        double s = 0.0;
        for (int k = tab[b] + threadIdx.x; k < tab[b + 1]; k += TPB) s += D.partials[c * total + k];
        sh[threadIdx.x] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            D.scal[b * B_NSCAL + slot + c] = (add_slot >= 0 ? D.scal[b * B_NSCAL + add_slot] : 0.0) + invN * sh[0];
        __syncthreads();
    }
}

// phi -= box mean (B_MEAN); PPT points per thread as in kb_sum
template <int PPT>
__global__ void __launch_bounds__(TPB) kb_sub_mean(BatchDev D, const int *__restrict__ tab, int fid, int active_only)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    const BoxDev &X = D.box[b];
    if (active_only && !D.active[b]) return;
    const int n = X.lev[0].n, N = n * n * n;
    const double mean = D.scal[b * B_NSCAL + B_MEAN];
    double *phi = X.field[fid];
    const int t0 = (blockIdx.x - tab[b]) * TPB * PPT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int t = t0 + q * TPB;
        if (t < N) phi[t] -= mean;
    }
}

// Stopping test per item of [b0, b1) (same criterion as the single-grid
// solver) and the cycle count; marks converged items inactive with the device
// clock time.  stall_ratio >= 0 (mixed precision): a refinement step that keeps
// more than that fraction of the previous relative residual counts as
// stalled, and two in a row stop the item's refinement with its fallback flag
// set (the host then finishes it with FP64 cycles, as the single grid does).
__global__ void kb_control(BatchDev D, int fid, double rtol, int max_cycles, int b0, int b1, double stall_ratio)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        if (!D.active[b]) continue;
        double *s = D.scal + b * B_NSCAL;
        const double rn = sqrt(s[B_RN]), fn = sqrt(s[B_FN]);
        const double rel = rn / (fn > 0.0 ? fn : 1.0);
        s[B_REL] = rel;
        int stop = 0;
        if (!isfinite(rel)) {
            D.status[b] = GR_ENAN;
            stop = 1;
        } else if (rtol > 0.0 && (rel <= rtol || rn == 0.0)) {
            stop = 1;
        } else if (D.cycles[b * 10 + fid] >= max_cycles) {
            if (rtol > 0.0) D.status[b] = GR_ENOTCONV;
            stop = 1;
        }
        if (!stop && stall_ratio >= 0.0) {
            s[B_STALL] = rel > stall_ratio * s[B_PREV] ? s[B_STALL] + 1.0 : 0.0;
            s[B_PREV] = rel;
            if (s[B_STALL] >= 2.0) {
                s[B_FB] = 1.0;
                D.active[b] = 0;
                continue;
            }
        }
        if (stop) {
            D.active[b] = 0;
            D.t_done[b * 10 + fid] = wall_clock64();
        } else {
            D.cycles[b * 10 + fid] += 1;
            atomicOr(&any, 1);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) *D.any_active = any;
}

// items [b0, b1) start solving field fid; clock slot ts (fid or 10 + fid)
__global__ void kb_begin_field(BatchDev D, int fid, int b0, int b1, int ts)
{
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        D.active[b] = 1;
        D.cycles[b * 10 + fid] = 0;
        double *s = D.scal + b * B_NSCAL;
        s[B_FBAR] = 0.0;
        s[B_FSHIFT] = 0.0;
        s[B_PREV] = HUGE_VAL;
        s[B_STALL] = 0.0;
        s[B_FB] = 0.0;
    }
    if (threadIdx.x == 0) D.t_start[ts] = wall_clock64();
}

// items of [b0, b1) whose mixed refinement stalled become the active set
// (set = 1), or every item inactive (set = 0); any_active reports the set
__global__ void kb_activate_fallback(BatchDev D, int b0, int b1, int set)
{
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        const int on = set && D.scal[b * B_NSCAL + B_FB] != 0.0;
        D.active[b] = on;
        if (on) atomicOr(&any, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *D.any_active = any;
}

// patches of [b0, b1) at nesting depth `depth` (all of them: depth < 0)
// become the active set
__global__ void kb_activate_depth(BatchDev D, int b0, int b1, int depth)
{
    for (int b = b0 + threadIdx.x; b < b1; b += blockDim.x) D.active[b] = depth < 0 || D.box[b].depth == depth;
}

// ------------------------------------------------------------- builders

// what: 0 V_i source (s_i - <s_i>) * 3 Om a with <s_i> in B_TMP, 1 -1/4 d.V,
// 2 A_ij/AA + Hamiltonian source + coefficient, 3 CMC coefficient/source,
// 4 shift sources, 5 -1/4 d.B, 6 copy fB[comp] to f
__global__ void __launch_bounds__(TPB) kb_build(BatchDev D, const int *__restrict__ tab, int what, int comp, double a,
                                                double om, double c)
{
    BOX_PROLOGUE(tab)
    const BoxLev &L = X.lev[0];
    const int n = L.n;
    if (t >= n * n * n) return;
    int x, y, z;
    decode3(t, n, n, x, y, z);
    const double inv2h = 1.0 / (2.0 * L.h);
    switch (what) {
    case 0: L.f[t] = (3.0 * om * a) * (X.src[1 + comp][t] - D.scal[b * B_NSCAL + B_TMP]); break;
    case 1: L.f[t] = div_quarter_point(X.field[GR_VX], X.field[GR_VY], X.field[GR_VZ], x, y, z, n, inv2h); break;
    case 2: {
        double A[6];
        const double aa = aij_point(X.field[GR_VX], X.field[GR_VY], X.field[GR_VZ], X.field[GR_U], x, y, z, n, L.h, A);
        for (int k = 0; k < 6; ++k) X.A6[k][t] = A[k];
        X.AA[t] = aa;
        L.coef[t] = aa;
        L.f[t] = (1.5 * a * om) * (X.src[0][t] - 1.0);
        break;
    }
    case 3: cmc_point(X.field[GR_PSI][t], X.src[0][t], X.src[4][t], X.AA[t], a, om, c, L.coef[t], L.f[t]); break;
    case 4: {
        double out[3];
        shift_source_point(X.field[GR_PSI], X.field[GR_XI], X.A6, x, y, z, n, L.h, a, c, out);
        X.fB[0][t] = out[0];
        X.fB[1][t] = out[1];
        X.fB[2][t] = out[2];
        break;
    }
    case 5: L.f[t] = div_quarter_point(X.field[GR_BX], X.field[GR_BY], X.field[GR_BZ], x, y, z, n, inv2h); break;
    default: L.f[t] = X.fB[comp][t]; break;
    }
}

__global__ void __launch_bounds__(TPB) kb_fill_field(BatchDev D, const int *__restrict__ tab, int fid)
{
    BOX_PROLOGUE(tab)
    const int n = X.lev[0].n;
    if (t < n * n * n) X.field[fid][t] = 0.0;
}

// ----------------------------------------------------- coarse cycle per box

template <int KIND>
__device__ void cvb_sweep(double *__restrict__ phi, const double *__restrict__ f, const double *__restrict__ coef, int n,
                          double inv_h2, OpConst oc, double Fb, double fs)
{
    const int half = n >> 1, tot = n * n * half;
    const SmallDiv dh(half), dn(n);
    for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < tot; t += CTPB) {
            const int r = dh.div(t), z = dn.div(r);
            const int x2 = t - r * half, y = r - z * n;
            const int i = 2 * x2 + ((y + z + colour) & 1);
            const long p = lin(i, y, z, n);
            const double ph = phi[p];
            double J;
            const double L = op_point<KIND, double>(ph, nb_sum(phi, i, y, z, n), inv_h2, load_c1<KIND>(coef, p), 0.0,
                                                    oc, Fb, J);
            phi[p] = ph - (L - (f[p] - fs)) / J;
        }
        __syncthreads();
    }
}

__device__ double cvb_block_sum(double v)
{
    __shared__ double sh[CTPB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < CTPB / 64; ++w) s += sh[w];
    __syncthreads();
    return s;
}

constexpr int kBoxCoarseLds = 1024; // doubles of LDS for the coarsest box level (8 KB)

template <int KIND>
__device__ void coarse_vcycle_box(const BatchDev &D, int b, int fid, int nu1, int nu2, OpConst oc)
{
    const BoxDev &X = D.box[b];
    const int l0 = X.centry, L = X.nlev;
    auto PHI = [&](int i) { return i == 0 ? X.field[fid] : X.lev[i].phi; };
    const double Fb0 = l0 == 0 ? D.scal[b * B_NSCAL + B_FBAR] : 0.0;
    const double fs0 = l0 == 0 ? D.scal[b * B_NSCAL + B_FSHIFT] : 0.0;
    for (int i = l0; i < L - 1; ++i) {
        const BoxLev &V = X.lev[i], &C = X.lev[i + 1];
        const int n = V.n, m = C.n;
        double *phi = PHI(i);
        const double inv_h2 = 1.0 / (V.h * V.h);
        const double Fb = i == 0 ? Fb0 : 0.0, fs = i == 0 ? fs0 : 0.0;
        for (int it = 0; it < nu1; ++it) cvb_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc, Fb, fs);
        const int M = m * m * m;
        for (int q = threadIdx.x; q < M; q += CTPB) {
            const int Xc = q % m, Yc = (q / m) % m, Zc = q / (m * m);
            double sr = 0.0, sp = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int a = 2 * Xc + (c & 1), bb = 2 * Yc + ((c >> 1) & 1), dd = 2 * Zc + (c >> 2);
                const long p = lin(a, bb, dd, n);
                const double ph = phi[p];
                double Jd;
                const double Lv = op_point<KIND, double>(ph, nb_sum(phi, a, bb, dd, n), inv_h2,
                                                         load_c1<KIND>(V.coef, p), 0.0, oc, Fb, Jd);
                sr += Lv - (V.f[p] - fs);
                sp += ph;
            }
            const double rp = sp / 8.0;
            C.phi[q] = rp;
            C.phi0[q] = rp;
            C.tmp[q] = sr / 8.0;
        }
        __syncthreads();
        const double inv_H2 = 1.0 / (C.h * C.h);
        for (int q = threadIdx.x; q < M; q += CTPB) {
            const int Xc = q % m, Yc = (q / m) % m, Zc = q / (m * m);
            double Jd;
            const double Lv = op_point<KIND, double>(C.phi[q], nb_sum(C.phi, Xc, Yc, Zc, m), inv_H2,
                                                     load_c1<KIND>(C.coef, q), 0.0, oc, 0.0, Jd);
            C.f[q] = Lv - C.tmp[q];
        }
        __syncthreads();
    }
    {
        const int i = L - 1;
        const BoxLev &V = X.lev[i];
        const int n = V.n, N = n * n * n;
        double *phi = PHI(i);
        const double inv_h2 = 1.0 / (V.h * V.h);
        const double Fb = i == 0 ? Fb0 : 0.0, fs = i == 0 ? fs0 : 0.0;
        for (int q = threadIdx.x; q < N; q += CTPB) V.tmp[q] = phi[q];
        __syncthreads();
        // the 32 sweeps from LDS when the level, its source and coefficient fit
        // (the coarsest box levels are 2^3 to 6^3), else from global memory
        constexpr int NC = kNumCoef<KIND>();
        __shared__ double lds[kBoxCoarseLds];
        if ((2 + NC) * N <= kBoxCoarseLds) {
            double *sphi = lds, *sf = lds + N, *sc = lds + 2 * N;
            for (int q = threadIdx.x; q < N; q += CTPB) {
                sphi[q] = phi[q];
                sf[q] = V.f[q];
                if (NC >= 1) sc[q] = V.coef[q];
            }
            __syncthreads();
            for (int it = 0; it < kCoarseSweeps; ++it) cvb_sweep<KIND>(sphi, sf, sc, n, inv_h2, oc, Fb, fs);
            for (int q = threadIdx.x; q < N; q += CTPB) phi[q] = sphi[q];
            __syncthreads();
        } else {
            for (int it = 0; it < kCoarseSweeps; ++it) cvb_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc, Fb, fs);
        }
        double dsum = 0.0;
        for (int q = threadIdx.x; q < N; q += CTPB) dsum += phi[q] - V.tmp[q];
        const double mean = cvb_block_sum(dsum) / (double)N;
        for (int q = threadIdx.x; q < N; q += CTPB) phi[q] -= mean;
        __syncthreads();
    }
    for (int i = L - 2; i >= l0; --i) {
        const BoxLev &V = X.lev[i], &C = X.lev[i + 1];
        const int n = V.n, m = C.n, N = n * n * n;
        double *phi = PHI(i);
        const double inv_h2 = 1.0 / (V.h * V.h);
        const double Fb = i == 0 ? Fb0 : 0.0, fs = i == 0 ? fs0 : 0.0;
        for (int p = threadIdx.x; p < N; p += CTPB) {
            const int a = p % n, bb = (p / n) % n, dd = p / (n * n);
            const int I = a >> 1, J = bb >> 1, K = dd >> 1;
            const int Is[2] = {I, wrapi(I + ((a & 1) ? 1 : -1), m)};
            const int Js[2] = {J, wrapi(J + ((bb & 1) ? 1 : -1), m)};
            const int Ks[2] = {K, wrapi(K + ((dd & 1) ? 1 : -1), m)};
            double v = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
                const long q = lin(Is[ox], Js[oy], Ks[oz], m);
                v += w * (C.phi[q] - C.phi0[q]);
            }
            phi[p] += v;
        }
        __syncthreads();
        for (int it = 0; it < nu2; ++it) cvb_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc, Fb, fs);
    }
}

template <int KIND>
__global__ void __launch_bounds__(CTPB) kb_coarse_vcycle(BatchDev D, int fid, int nu1, int nu2, OpConst oc)
{
    if (!D.active[blockIdx.x]) return;
    coarse_vcycle_box<KIND>(D, blockIdx.x, fid, nu1, nu2, oc);
}

// ------------------------------------------------ persistent task queue
//
// One launch per V-cycle runs, for every active box, its levels from the
// queue entry (the first level of at most queue_n^3 points) down to the
// single-workgroup coarse cycle and back up.  Tasks (item, level, phase,
// z-range) are taken in table order from a device-wide ticket; the table lists
// the phases of all items phase-major, each phase split into z-ranges of
// about kQTarget points.  A task first waits until its item's counter of
// completed tasks reaches the number of the item's tasks in earlier phases,
// so one item's phases run in order while items and z-ranges run in parallel.
// A worker only ever waits on tasks with smaller tickets, which running
// workers already hold, so the queue drains whatever the residency.  Every
// wait is bounded: on a timeout the item's status becomes GR_EDEVICE and the
// queue's abort flag makes all later tasks skip.  Data written by one task
// and read by a later one (possibly on another XCD) is published by thread 0's
// agent-scope release increment after a workgroup barrier, and acquired by the
// waiting thread 0's agent-scope acquire load before a barrier (the pattern of
// a grid-wide barrier).
enum QPhase { Q_RED = 0, Q_BLACK = 1, Q_RR = 2, Q_CRHS = 3, Q_PROLONG = 4, Q_COARSE = 5 };
struct QTask {
    int item, phase, level, z0, z1, prefix;
};
constexpr int kQTarget = 4096;  // points per task (default; GRMG_QUEUE_TARGET)
constexpr int kQueueMaxNu = 8;  // task table capacity: nu1, nu2 <= 8
constexpr long kQSpin = 1L << 22; // bounded wait (iterations of a short sleep)

// ctl[0]: ticket, ctl[1]: abort (full = 1 also clears it); done[item] = 0
__global__ void kb_queue_reset(int *__restrict__ ctl, int *__restrict__ done, int nbox, int full)
{
    for (int b = threadIdx.x; b < nbox; b += blockDim.x) done[b] = 0;
    if (threadIdx.x == 0) {
        ctl[0] = 0;
        if (full) ctl[1] = 0;
    }
}

template <int KIND>
__device__ void q_run(const BatchDev &D, const QTask &q, int fid, int nu1, int nu2, OpConst oc)
{
    const int b = q.item, i = q.level;
    if (q.phase == Q_COARSE) {
        coarse_vcycle_box<KIND>(D, b, fid, nu1, nu2, oc);
        return;
    }
    const BoxDev &X = D.box[b];
    const BoxLev &V = X.lev[i];
    const int n = V.n;
    double *phi = i == 0 ? X.field[fid] : V.phi;
    const double Fb = i == 0 ? D.scal[b * B_NSCAL + B_FBAR] : 0.0;
    const double fs = i == 0 ? D.scal[b * B_NSCAL + B_FSHIFT] : 0.0;
    if (q.phase == Q_RED || q.phase == Q_BLACK) { // one colour of planes z0..z1 (as kb_colour)
        const int colour = q.phase, half = n >> 1, tot = (q.z1 - q.z0) * n * half;
        const double inv_h2 = 1.0 / (V.h * V.h);
        for (int t = threadIdx.x; t < tot; t += CTPB) {
            const int x2 = t % half, r = t / half, y = r % n, z = q.z0 + r / n;
            const int ii = 2 * x2 + ((y + z + colour) & 1);
            const long p = lin(ii, y, z, n);
            const double ph = phi[p];
            double J;
            const double Lv = op_point<KIND, double>(ph, nb_sum(phi, ii, y, z, n), inv_h2, load_c1<KIND>(V.coef, p),
                                                     0.0, oc, Fb, J);
            phi[p] = ph - (Lv - (V.f[p] - fs)) / J;
        }
        return;
    }
    const BoxLev &C = X.lev[i + 1];
    const int m = C.n;
    if (q.phase == Q_RR) { // residual + restriction into coarse planes z0..z1 (as kb_rr_m per cell)
        const int tot = (q.z1 - q.z0) * m * m;
        const double inv_h2 = 1.0 / (V.h * V.h);
        for (int t = threadIdx.x; t < tot; t += CTPB) {
            const int I = t % m, J = (t / m) % m, K = q.z0 + t / (m * m);
            double sr = 0.0, sp = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int a = 2 * I + (c & 1), bb = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
                const long p = lin(a, bb, k, n);
                const double ph = phi[p];
                double Jd;
                const double Lv = op_point<KIND, double>(ph, nb_sum(phi, a, bb, k, n), inv_h2,
                                                         load_c1<KIND>(V.coef, p), 0.0, oc, Fb, Jd);
                sr += Lv - (V.f[p] - fs);
                sp += ph;
            }
            const long c0 = lin(I, J, K, m);
            const double rp = sp / 8.0;
            C.phi[c0] = rp;
            C.phi0[c0] = rp;
            C.tmp[c0] = sr / 8.0;
        }
    } else if (q.phase == Q_CRHS) { // FAS source of coarse planes z0..z1 (as kb_coarse_rhs)
        const int tot = (q.z1 - q.z0) * m * m;
        const double inv_H2 = 1.0 / (C.h * C.h);
        for (int t = threadIdx.x; t < tot; t += CTPB) {
            const int I = t % m, J = (t / m) % m, K = q.z0 + t / (m * m);
            const long c0 = lin(I, J, K, m);
            double Jd;
            const double Lv = op_point<KIND, double>(C.phi[c0], nb_sum(C.phi, I, J, K, m), inv_H2,
                                                     load_c1<KIND>(C.coef, c0), 0.0, oc, 0.0, Jd);
            C.f[c0] = Lv - C.tmp[c0];
        }
    } else { // Q_PROLONG: fine planes z0..z1 += P (phi^H - phi0^H), the coarse cycle's per-point form
        const int tot = (q.z1 - q.z0) * n * n;
        for (int t = threadIdx.x; t < tot; t += CTPB) {
            const int a = t % n, bb = (t / n) % n, dd = q.z0 + t / (n * n);
            const int I = a >> 1, J = bb >> 1, K = dd >> 1;
            const int Is[2] = {I, wrapi(I + ((a & 1) ? 1 : -1), m)};
            const int Js[2] = {J, wrapi(J + ((bb & 1) ? 1 : -1), m)};
            const int Ks[2] = {K, wrapi(K + ((dd & 1) ? 1 : -1), m)};
            double v = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
                const long qq = lin(Is[ox], Js[oy], Ks[oz], m);
                v += w * (C.phi[qq] - C.phi0[qq]);
            }
            phi[lin(a, bb, dd, n)] += v;
        }
    }
}

template <int KIND>
__global__ void __launch_bounds__(CTPB) kb_queue(BatchDev D, const QTask *__restrict__ tasks, int ntasks,
                                                 int *__restrict__ ctl, int *__restrict__ done, int fid, int nu1,
                                                 int nu2, OpConst oc, long spin_limit)
{
    __shared__ int s_t, s_go;
    for (;;) {
        if (threadIdx.x == 0) {
            const int t = atomicAdd(&ctl[0], 1);
            int go = 0;
            if (t < ntasks) {
                const QTask q = tasks[t];
                if (D.active[q.item] && !__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    go = 1;
                    long it = 0;
                    while (__hip_atomic_load(&done[q.item], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < q.prefix) {
                        if (++it > spin_limit || __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            if (it > spin_limit) D.status[q.item] = GR_EDEVICE;
                            __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            go = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
            }
            s_t = t;
            s_go = go;
        }
        __syncthreads();
        const int t = s_t, go = s_go;
        if (t >= ntasks) return;
        if (go) { // thread 0's acquire, then the barrier, orders every thread's reads after the wait
            const QTask q = tasks[t];
            q_run<KIND>(D, q, fid, nu1, nu2, oc);
            __syncthreads(); // every thread's writes before thread 0's release
            if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[q.item], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads(); // s_t, s_go are rewritten next
    }
}

// ------------------------------------------- mixed precision (periodic boxes)
//
// Iterative refinement as on a single grid: the FP64 residual of the
// regularised fine equation (with the cycle's frozen means) becomes the FP32
// source b = -r of the linearised correction equation J e = b, which one FP32
// V-cycle solves approximately (coarse levels from 8^3 down in FP64, in LDS,
// one workgroup per box); then phi += e - <e> in FP64.

// FP64 residual -> b (FP32), the frozen Hamiltonian linearisation a = chi and
// c = dL/dPsi + 6 chi/h^2, and block partials of r^2 and (f - fshift)^2
// (the norms table's block layout: the plane-marching form for the boxes it
// marches, one thread per point for the others)
template <int KIND>
__global__ void __launch_bounds__(TPB) kb_ir_m(BatchDev D, const int *__restrict__ tab, int fid, OpConst oc)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    const BoxDev &X = D.box[b];
    const int total = tab[D.nbox];
    const int lb = blockIdx.x - tab[b];
    const BoxLev &L = X.lev[0];
    const int n = L.n;
    double v[2] = {0.0, 0.0};
    if (D.active[b]) {
        const double Fb = D.scal[b * B_NSCAL + B_FBAR], fs = D.scal[b * B_NSCAL + B_FSHIFT];
        const double inv_h2 = 1.0 / (L.h * L.h);
        const double *phi = X.field[fid];
        if (D.march && marchable(n)) { // the block table gives march_blocks(n) blocks
            const int mz = mz_chunk(n), nzc = n / mz, tiles_y = n / MTY, tile = lb / nzc, zchunk = lb % nzc;
            march_tile<M_IR, KIND, double>(phi, L.f, L.coef, nullptr, n, mz, inv_h2, oc, Fb, fs,
                                           (tile / tiles_y) * MTX, (tile % tiles_y) * MTY, zchunk * mz, nullptr,
                                           nullptr, nullptr, L.b32, L.a32, L.c32, v);
        } else {
            const int t = lb * TPB + threadIdx.x;
            if (t < n * n * n) {
                int x, y, z;
                decode3(t, n, n, x, y, z);
                const double ph = phi[t];
                double J;
                const double Lv = op_point<KIND, double>(ph, nb_sum(phi, x, y, z, n), inv_h2,
                                                         load_c1<KIND>(L.coef, t), 0.0, oc, Fb, J);
                const double fe = L.f[t] - fs;
                const double e = Lv - fe;
                v[0] = e * e;
                v[1] = fe * fe;
                L.b32[t] = (float)(-e);
                if constexpr (KIND == GR_KIND_HAMILTONIAN) {
                    const double chi = 1.0 - oc.kappa * ph;
                    L.a32[t] = (float)chi;
                    L.c32[t] = (float)(J + 6.0 * chi * inv_h2);
                }
            }
        }
    }
    block_store<2>(v, D.partials, total);
}

// c = -m2 in FP32 on the finest level (linearised CMC coefficient)
__global__ void __launch_bounds__(TPB) kb_neg_coef32(BatchDev D, const int *__restrict__ tab)
{
    BOX_PROLOGUE(tab)
    const BoxLev &L = X.lev[0];
    if (t < L.n * L.n * L.n) L.c32[t] = (float)(-L.coef[t]);
}

// FP32 restriction of the linearisation, level d -> d+1 (which: 0 c, 1 a)
__global__ void __launch_bounds__(TPB) kb_restrict32(BatchDev D, const int *__restrict__ tab, int d, int which)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int m = C.n, n = V.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    const float *src = which ? V.a32 : V.c32;
    float s = 0.f;
    for (int c = 0; c < 8; ++c) s += src[lin(2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2), n)];
    (which ? C.a32 : C.c32)[t] = s / 8.f;
}

// (fine8 table: kSumPPT points per thread)
__global__ void __launch_bounds__(TPB) kb32_fill(BatchDev D, const int *__restrict__ tab, int d)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    if (!D.active[b]) return;
    const BoxLev &L = D.box[b].lev[d];
    const int N = L.n * L.n * L.n, t0 = (blockIdx.x - tab[b]) * TPB * kSumPPT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kSumPPT; ++q)
        if (t0 + q * TPB < N) L.e[t0 + q * TPB] = 0.f;
}

// one colour of a red-black sweep of the correction equation on level d
template <int LKIND>
__global__ void __launch_bounds__(TPB) kb32_colour(BatchDev D, const int *__restrict__ tab, int d, int colour,
                                                   OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &L = X.lev[d];
    const int n = L.n, half = n >> 1;
    if (t >= n * n * half) return;
    int x2, y, z;
    decode3(t, half, n, x2, y, z);
    const int i = 2 * x2 + ((y + z + colour) & 1);
    const long p = lin(i, y, z, n);
    const float ph = L.e[p];
    const float ih2 = (float)(1.0 / (L.h * L.h));
    float J;
    const float Lv = op_point<LKIND, float>(ph, nb_sum(L.e, i, y, z, n), ih2, load_c1<LKIND>(L.c32, p),
                                            load_c2<LKIND>(L.a32, p), oc, 0.f, J);
    L.e[p] = newton_update<LKIND, float>(ph, Lv, L.b32[p], J, poisson_inv_diag(ih2));
}

// fused red-black sweeps of the correction equation (rb_fused_tile in FP32)
// for the boxes whose level d takes fused tiles: even sweeps e -> t32, odd
// t32 -> e
template <int LKIND, int TX, int TY>
__global__ void __launch_bounds__((TX / 2) * TY) kb32_fused(BatchDev D, const int *__restrict__ tab, int d, int sweep,
                                                            OpConst oc)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const BoxLev &L = X.lev[d];
    const int n = L.n, lb = blockIdx.x - tab[b];
    const int nz = n / kFZ, tiles_y = n / TY;
    const int zchunk = lb % nz, t2 = lb / nz;
    const float *in = (sweep & 1) ? L.t32 : L.e;
    float *out = (sweep & 1) ? L.e : L.t32;
    rb_fused_tile<LKIND, float, TX, TY, 2>(in, out, L.b32, L.c32, L.a32, n, kFZ, (float)(1.0 / (L.h * L.h)), oc, 0.f,
                                           0.f, (t2 / tiles_y) * TX, (t2 % tiles_y) * TY, zchunk * kFZ);
}

// coarse source b^H = R(b - J e) and e^H = 0: one thread per cell of level d+1
template <int LKIND>
__global__ void __launch_bounds__(TPB) kb32_lin_rr(BatchDev D, const int *__restrict__ tab, int d, OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int n = V.n, m = C.n;
    const float inv_h2 = (float)(1.0 / (V.h * V.h));
    if (D.march && marchable(n)) { // the block table gives march_blocks(n) blocks
        const int lb = blockIdx.x - tab[b];
        const int mz = mz_chunk(n), nzc = n / mz, tiles_y = n / MTY, tile = lb / nzc, zchunk = lb % nzc;
        double v[2];
        march_tile<M_RESTRICT_LIN, LKIND, float>(V.e, V.b32, V.c32, V.a32, n, mz, inv_h2, oc, 0.f, 0.f,
                                                 (tile / tiles_y) * MTX, (tile % tiles_y) * MTY, zchunk * mz, C.b32,
                                                 C.e, nullptr, nullptr, nullptr, nullptr, v);
        return;
    }
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    float sr = 0.f;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
        const long p = lin(i, j, k, n);
        float Jd;
        const float Lv = op_point<LKIND, float>(V.e[p], nb_sum(V.e, i, j, k, n), inv_h2, load_c1<LKIND>(V.c32, p),
                                                load_c2<LKIND>(V.a32, p), oc, 0.f, Jd);
        sr += V.b32[p] - Lv;
    }
    C.b32[t] = sr / 8.f;
    C.e[t] = 0.f;
}

// e^h += P e^H (cell-centred trilinear, periodic): one thread per coarse cell,
// which reads its 3^3 coarse neighbourhood once and updates its 8 children
// (each child sums its 8 coarse neighbours in the same order as the FP64 form)
__global__ void __launch_bounds__(TPB) kb32_prolong(BatchDev D, const int *__restrict__ tab, int d)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int n = V.n, m = C.n;
    if (t >= m * m * m) return;
    int x, y, z;
    decode3(t, m, m, x, y, z);
    float e[3][3][3];
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                e[dz + 1][dy + 1][dx + 1] = C.e[lin(wrapi(x + dx, m), wrapi(y + dy, m), wrapi(z + dz, m), m)];
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy) {
            float v[2];
            for (int cx = 0; cx < 2; ++cx) {
                const int sx = cx ? 1 : -1, sy = cy ? 1 : -1, sz = cz ? 1 : -1;
                float a = 0.f;
                for (int c = 0; c < 8; ++c) {
                    const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                    const float w = (ox ? 0.25f : 0.75f) * (oy ? 0.25f : 0.75f) * (oz ? 0.25f : 0.75f);
                    a += w * e[1 + oz * sz][1 + oy * sy][1 + ox * sx];
                }
                v[cx] = a;
            }
            float2 *dst = reinterpret_cast<float2 *>(V.e + lin(2 * x, 2 * y + cy, 2 * z + cz, n));
            float2 old = *dst;
            old.x += v[0];
            old.y += v[1];
            *dst = old;
        }
}

// the correction cycle from the box's FP32 entry level down, one workgroup per
// box, computed in FP64 in LDS
template <int LKIND>
__global__ void __launch_bounds__(kCoarseThreads) kb32_coarse(BatchDev D, int nu1, int nu2, OpConst oc)
{
    const int b = blockIdx.x;
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    CoarseLevelsT<float> G;
    G.nl = X.nlev - X.centry32;
    for (int i = 0; i < G.nl; ++i) {
        const BoxLev &V = X.lev[X.centry32 + i];
        G.n[i] = V.n;
        G.inv_h2[i] = 1.0 / (V.h * V.h);
        G.phi[i] = V.e;
        G.phi0[i] = nullptr;
        G.f[i] = V.b32;
        G.c1[i] = V.c32;
        G.c2[i] = V.a32;
        G.tmp[i] = V.t32;
    }
    const double *zero = D.scal + b * B_NSCAL + B_ZERO;
    coarse_cycle_lds<LKIND, float, double>(G, nu1, nu2, oc, zero, zero);
}

// phi += e - <e> (mean in B_MEAN), FP64
// (fine8 table: kSumPPT points per thread)
__global__ void __launch_bounds__(TPB) kb_ir_update(BatchDev D, const int *__restrict__ tab, int fid)
{
    const int b = find_box(tab, D.nbox, blockIdx.x);
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const BoxLev &L = X.lev[0];
    const double mean = D.scal[b * B_NSCAL + B_MEAN];
    double *phi = X.field[fid];
    const int N = L.n * L.n * L.n, t0 = (blockIdx.x - tab[b]) * TPB * kSumPPT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kSumPPT; ++q) {
        const int t = t0 + q * TPB;
        if (t < N) phi[t] += (double)L.e[t] - mean;
    }
}

// ------------------------------------------------- Dirichlet patches
//
// Same phases as the periodic boxes, one launch per phase over all patches
// (prefix tables over the patch items), one thread per cell.  Iterate arrays
// are padded (patch_ops.h); everything else is dense n^3.

__device__ __forceinline__ double *patch_phi(const BoxDev &X, int d, int fid)
{
    return d == 0 ? X.field[fid] : X.lev[d].phi;
}

template <int KIND>
__global__ void __launch_bounds__(TPB) kp_colour(BatchDev D, const int *__restrict__ tab, int d, int fid, int colour,
                                                 OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &L = X.lev[d];
    const int n = L.n, half = n >> 1; // grouped patch levels have even n
    if (t >= n * n * half) return;
    int x2, j, k;
    decode3(t, half, n, x2, j, k);
    const int i = 2 * x2 + ((j + k + colour) & 1);
    double *phi = patch_phi(X, d, fid);
    double J;
    const long q = lin(i, j, k, n);
    const double Lv = patch_op<KIND>(phi, i, j, k, n, 1.0 / (L.h * L.h), load_c1<KIND>(L.coef, q), oc, J);
    const long p = pidx(i, j, k, n);
    phi[p] = phi[p] - (Lv - L.f[q]) / J;
}

// Fused red-black sweep of patch levels: one workgroup per TX x TY x TZ tile
// of a level.  The tile's neighbourhood with a 2-cell halo (the face values b
// in the padded layer included) is read into LDS; red points of the tile and of
// its 1-cell ring are updated from old values, then the tile's black points
// from those, and the tile is written out of place (even sweeps phi -> ptmp,
// odd ptmp -> phi), so tiles never read each other's output and the result is
// the red-then-black sweep of kp_colour.  Boundary cells use 2b - phi_cell
// across their faces with the matching Newton derivative; the Poisson kinds
// multiply by the constant -1/J = h^2/(6 + faces) instead of dividing.
__constant__ const double kInvDiag[4] = {1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0, 1.0 / 9.0}; // 1/(6 + boundary faces)

template <int KIND>
__device__ __forceinline__ double patch_op_lds(const double *__restrict__ s, int q, int W, int W2, int i, int j, int k,
                                               int n, double inv_h2, double c1, OpConst oc, double &J, int &nf)
{
    const double ph = s[q];
    double nbs = s[q - 1] + s[q + 1] + s[q - W] + s[q + W] + s[q - W2] + s[q + W2];
    nf = 0;
    if (i == 0) { nbs += s[q - 1] - ph; ++nf; }
    if (i == n - 1) { nbs += s[q + 1] - ph; ++nf; }
    if (j == 0) { nbs += s[q - W] - ph; ++nf; }
    if (j == n - 1) { nbs += s[q + W] - ph; ++nf; }
    if (k == 0) { nbs += s[q - W2] - ph; ++nf; }
    if (k == n - 1) { nbs += s[q + W2] - ph; ++nf; }
    const double L = op_point<KIND, double>(ph, nbs, inv_h2, c1, 0.0, oc, 0.0, J);
    if (nf) J -= (double)nf * inv_h2 * (KIND == GR_KIND_HAMILTONIAN ? 1.0 - oc.kappa * ph : 1.0);
    return L;
}

template <int KIND, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TPB) kp_fused(BatchDev D, const int *__restrict__ tab, int d, int fid, int sweep,
                                                OpConst oc)
{
    constexpr int HX = TX + 4, HY = TY + 4, HZ = TZ + 4, RX = TX + 2, RY = TY + 2, RZ = TZ + 2;
    __shared__ double s_old[HX * HY * HZ];
    __shared__ double s_red[RX * RY * RZ];
    // XCD-contiguous order: the grid is a multiple of 8 and block g (on XCD
    // g mod 8) takes tile v, so every XCD sweeps one contiguous run of tiles
    // and neighbouring tiles share their halos in that XCD's L2
    const int per = gridDim.x >> 3, v = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (v >= tab[D.nbox]) return;
    const int b = find_box(tab, D.nbox, v);
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const BoxLev &L = X.lev[d];
    const int n = L.n, ntx = (n + TX - 1) / TX, nty = (n + TY - 1) / TY, lb = v - tab[b];
    const int ox = (lb % ntx) * TX, oy = ((lb / ntx) % nty) * TY, oz = (lb / (ntx * nty)) * TZ;
    double *phi = patch_phi(X, d, fid);
    const double *in = (sweep & 1) ? L.ptmp : phi;
    double *out = (sweep & 1) ? phi : L.ptmp;
    const double inv_h2 = 1.0 / (L.h * L.h), h2 = L.h * L.h;
    // old values of the 12^3 neighbourhood (cells beyond the padded layer are never used)
    for (int t = threadIdx.x; t < HX * HY * HZ; t += TPB) {
        const int a = t % HX, c = (t / HX) % HY, e = t / (HX * HY);
        const int i = ox - 2 + a, j = oy - 2 + c, k = oz - 2 + e;
        const bool in_pad = i >= -1 && i <= n && j >= -1 && j <= n && k >= -1 && k <= n;
        s_old[t] = in_pad ? in[pidx(i, j, k, n)] : 0.0;
    }
    __syncthreads();
    // red points of the tile and its ring from old values; every other cell keeps its old value
    for (int t = threadIdx.x; t < RX * RY * RZ; t += TPB) {
        const int a = t % RX, c = (t / RX) % RY, e = t / (RX * RY);
        const int i = ox - 1 + a, j = oy - 1 + c, k = oz - 1 + e;
        const int q = ((e + 1) * HY + (c + 1)) * HX + (a + 1);
        double v = s_old[q];
        if (i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n && ((i + j + k) & 1) == 0) {
            double J;
            int nf;
            const long g = lin(i, j, k, n);
            const double Lv = patch_op_lds<KIND>(s_old, q, HX, HX * HY, i, j, k, n, inv_h2, load_c1<KIND>(L.coef, g),
                                                 oc, J, nf);
            v = KIND == GR_KIND_POISSON ? v + (Lv - L.f[g]) * (h2 * kInvDiag[nf]) : v - (Lv - L.f[g]) / J;
        }
        s_red[t] = v;
    }
    __syncthreads();
    // black points of the tile from the updated red values; the tile written out
    for (int t = threadIdx.x; t < TX * TY * TZ; t += TPB) {
        const int a = t % TX, c = (t / TX) % TY, e = t / (TX * TY);
        const int i = ox + a, j = oy + c, k = oz + e;
        if (i >= n || j >= n || k >= n) continue;
        const int q = ((e + 1) * RY + (c + 1)) * RX + (a + 1);
        double v = s_red[q];
        if (((i + j + k) & 1) == 1) {
            double J;
            int nf;
            const long g = lin(i, j, k, n);
            const double Lv = patch_op_lds<KIND>(s_red, q, RX, RX * RY, i, j, k, n, inv_h2, load_c1<KIND>(L.coef, g),
                                                 oc, J, nf);
            v = KIND == GR_KIND_POISSON ? v + (Lv - L.f[g]) * (h2 * kInvDiag[nf]) : v - (Lv - L.f[g]) / J;
        }
        out[pidx(i, j, k, n)] = v;
    }
}

// residual at the 8 children, its mean, and the children's mean of phi (R phi,
// also kept as phi0): one thread per interior cell of level d+1
template <int KIND>
__global__ void __launch_bounds__(TPB) kp_rr(BatchDev D, const int *__restrict__ tab, int d, int fid, OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int n = V.n, m = C.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    const double *phi = patch_phi(X, d, fid);
    const double inv_h2 = 1.0 / (V.h * V.h);
    double sr = 0.0, sp = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
        const long q = lin(i, j, k, n);
        double Jd;
        sr += patch_op<KIND>(phi, i, j, k, n, inv_h2, load_c1<KIND>(V.coef, q), oc, Jd) - V.f[q];
        sp += phi[pidx(i, j, k, n)];
    }
    const double rp = sp / 8.0;
    C.phi[pidx(I, J, K, m)] = rp;
    C.phi0[t] = rp;
    C.tmp[t] = sr / 8.0;
}

// FAS source of level d+1: f^H = L^H(R phi) - R eps, with the level's face values
template <int KIND>
__global__ void __launch_bounds__(TPB) kp_coarse_rhs(BatchDev D, const int *__restrict__ tab, int d, OpConst oc)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &C = X.lev[d + 1];
    const int m = C.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    double Jd;
    C.f[t] = patch_op<KIND>(C.phi, I, J, K, m, 1.0 / (C.h * C.h), load_c1<KIND>(C.coef, t), oc, Jd) - C.tmp[t];
}

// phi^h += P(phi^H - R phi), the correction odd across every face: one
// thread per interior cell of level d
__global__ void __launch_bounds__(TPB) kp_prolong(BatchDev D, const int *__restrict__ tab, int d, int fid)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int n = V.n, m = C.n;
    if (t >= n * n * n) return;
    int i, j, k;
    decode3(t, n, n, i, j, k);
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int Is[2] = {I, I + ((i & 1) ? 1 : -1)};
    const int Js[2] = {J, J + ((j & 1) ? 1 : -1)};
    const int Ks[2] = {K, K + ((k & 1) ? 1 : -1)};
    double v = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
        const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
        double sign = 1.0;
        const int x = reflect_in(Is[ox], m, sign), y = reflect_in(Js[oy], m, sign), z = reflect_in(Ks[oz], m, sign);
        v += w * (sign * (C.phi[pidx(x, y, z, m)] - C.phi0[lin(x, y, z, m)]));
    }
    patch_phi(X, d, fid)[pidx(i, j, k, n)] += v;
}

// coefficient restriction level d -> d+1 (once per solve of an equation)
__global__ void __launch_bounds__(TPB) kp_restrict_coef(BatchDev D, const int *__restrict__ tab, int d)
{
    BOX_PROLOGUE(tab)
    const BoxLev &V = X.lev[d], &C = X.lev[d + 1];
    const int m = C.n, n = V.n;
    if (t >= m * m * m) return;
    int I, J, K;
    decode3(t, m, m, I, J, K);
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += V.coef[lin(2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2), n)];
    C.coef[t] = s / 8.0;
}

// stopping norms of the finest level: block partials of eps^2 and f^2
template <int KIND>
__global__ void __launch_bounds__(TPB) kp_norms(BatchDev D, const int *__restrict__ tab, int fid, OpConst oc)
{
    BOX_PROLOGUE(tab)
    const int total = tab[D.nbox];
    const BoxLev &L = X.lev[0];
    const int n = L.n;
    double v[2] = {0.0, 0.0};
    if (D.active[b] && t < n * n * n) {
        int i, j, k;
        decode3(t, n, n, i, j, k);
        double Jd;
        const double e = patch_op<KIND>(X.field[fid], i, j, k, n, 1.0 / (L.h * L.h), load_c1<KIND>(L.coef, t), oc,
                                        Jd) - L.f[t];
        v[0] = e * e;
        v[1] = L.f[t] * L.f[t];
    }
    block_store<2>(v, D.partials, total);
}

// boundary values of level d of every patch: the parent's field `fid` at the
// face centres, one thread per padded cell (face cells written; edge and
// corner cells are never read)
__global__ void __launch_bounds__(TPB) kp_faces(BatchDev D, const int *__restrict__ tab, int d, int fid)
{
    BOX_PROLOGUE(tab)
    if (!D.active[b]) return;
    const BoxLev &L = X.lev[d];
    const int n = L.n, W = n + 2;
    if (t >= W * W * W) return;
    int a, bb, c;
    decode3(t, W, W, a, bb, c);
    const int i = a - 1, j = bb - 1, k = c - 1;
    const int out = (i < 0 || i >= n) + (j < 0 || j >= n) + (k < 0 || k >= n);
    if (out != 1) return;
    auto u = [n](int q) { return q < 0 ? 0.0 : (q >= n ? (double)n : q + 0.5); }; // face-clamped coordinate
    const BoxDev &P = D.box[X.parent];
    const double val = sample_parent_at(P.field[fid], P.patch, 1, P.lev[0].n, P.lev[0].h, X.origin[0] + u(i) * L.h,
                                        X.origin[1] + u(j) * L.h, X.origin[2] + u(k) * L.h);
    patch_phi(X, d, fid)[t] = val;
    if (L.ptmp) L.ptmp[t] = val;
}

// interior := 0 (zero guess)
__global__ void __launch_bounds__(TPB) kp_fill_field(BatchDev D, const int *__restrict__ tab, int fid)
{
    BOX_PROLOGUE(tab)
    const int n = X.lev[0].n;
    if (t >= n * n * n) return;
    int i, j, k;
    decode3(t, n, n, i, j, k);
    X.field[fid][pidx(i, j, k, n)] = 0.0;
}

// Source builders of the patches, the periodic builders' arithmetic through
// patch field accessors (outside the patch: the parent's field at the cell
// centre).  what: 0 V_i source 3 Om a s_i (no mean removed), 1 -1/4 d.V,
// 2 A_ij/AA + Hamiltonian source + coefficient, 3 CMC coefficient/source,
// 4 shift sources, 5 -1/4 d.B, 6 copy fB[comp] to f
__global__ void __launch_bounds__(TPB) kp_build(BatchDev D, const int *__restrict__ tab, int what, int comp, double a,
                                                double om, double c)
{
    BOX_PROLOGUE(tab)
    const BoxLev &L = X.lev[0];
    const int n = L.n;
    if (t >= n * n * n) return;
    int x, y, z;
    decode3(t, n, n, x, y, z);
    const BoxDev &P = D.box[X.parent];
    // the parent's fields are padded when it is a patch; its A_ij is dense
    auto F = [&](const double *mine, int padded, const double *theirs, int ppadded) {
        return PatchField{mine, padded, n, L.h, X.origin[0], X.origin[1], X.origin[2], theirs, P.lev[0].n, P.lev[0].h,
                          P.patch, ppadded};
    };
    auto FF = [&](int f) { return F(X.field[f], 1, P.field[f], 1); };
    const double inv2h = 1.0 / (2.0 * L.h);
    switch (what) {
    case 0: L.f[t] = (3.0 * om * a) * X.src[1 + comp][t]; break;
    case 1: L.f[t] = div_quarter_f(FF(GR_VX), FF(GR_VY), FF(GR_VZ), x, y, z, inv2h); break;
    case 2: {
        double A[6];
        const double aa = aij_f(FF(GR_VX), FF(GR_VY), FF(GR_VZ), FF(GR_U), x, y, z, L.h, A);
        for (int k = 0; k < 6; ++k) X.A6[k][t] = A[k];
        X.AA[t] = aa;
        L.coef[t] = aa;
        L.f[t] = (1.5 * a * om) * (X.src[0][t] - 1.0);
        break;
    }
    case 3:
        cmc_point(X.field[GR_PSI][pidx(x, y, z, n)], X.src[0][t], X.src[4][t], X.AA[t], a, om, c, L.coef[t], L.f[t]);
        break;
    case 4: {
        const PatchField A[6] = {F(X.A6[0], 0, P.A6[0], 0), F(X.A6[1], 0, P.A6[1], 0), F(X.A6[2], 0, P.A6[2], 0),
                                 F(X.A6[3], 0, P.A6[3], 0), F(X.A6[4], 0, P.A6[4], 0), F(X.A6[5], 0, P.A6[5], 0)};
        double out[3];
        shift_source_f(FF(GR_PSI), FF(GR_XI), A, x, y, z, L.h, a, c, out);
        X.fB[0][t] = out[0];
        X.fB[1][t] = out[1];
        X.fB[2][t] = out[2];
        break;
    }
    case 5: L.f[t] = div_quarter_f(FF(GR_BX), FF(GR_BY), FF(GR_BZ), x, y, z, inv2h); break;
    default: L.f[t] = X.fB[comp][t]; break;
    }
}

// dense n^3 <-> interior of a padded (n+2)^3 array
template <typename T>
__global__ void __launch_bounds__(TPB) kp_pad_in(double *__restrict__ dst, const T *__restrict__ src, int n)
{
    const long t = (long)blockIdx.x * TPB + threadIdx.x;
    if (t >= (long)n * n * n) return;
    int i, j, k;
    decode3((int)t, n, n, i, j, k);
    dst[pidx(i, j, k, n)] = (double)src[t];
}
template <typename T>
__global__ void __launch_bounds__(TPB) kp_pad_out(T *__restrict__ dst, const double *__restrict__ src, int n)
{
    const long t = (long)blockIdx.x * TPB + threadIdx.x;
    if (t >= (long)n * n * n) return;
    int i, j, k;
    decode3((int)t, n, n, i, j, k);
    dst[t] = (T)src[pidx(i, j, k, n)];
}

// The rest of the V-cycle of each active patch from its entry level, one
// workgroup per patch (item b0 + blockIdx.x).
template <int KIND>
__device__ void cvp_sweep(double *__restrict__ phi, const double *__restrict__ f, const double *__restrict__ coef,
                          int n, double inv_h2, OpConst oc)
{
    const int N = n * n * n;
    const SmallDiv dn(n);
    for (int colour = 0; colour < 2; ++colour) {
        for (int t = threadIdx.x; t < N; t += CTPB) {
            const int r = dn.div(t), k = dn.div(r);
            const int i = t - r * n, j = r - k * n;
            if (((i + j + k) & 1) != colour) continue;
            double J;
            const double Lv = patch_op<KIND>(phi, i, j, k, n, inv_h2, load_c1<KIND>(coef, t), oc, J);
            const long p = pidx(i, j, k, n);
            phi[p] = phi[p] - (Lv - f[t]) / J;
        }
        __syncthreads();
    }
}

constexpr int kPatchCoarseLds = 4096; // doubles of LDS for the coarsest patch level (32 KB)

template <int KIND>
__global__ void __launch_bounds__(CTPB) kp_coarse_vcycle(BatchDev D, int fid, int nu1, int nu2, OpConst oc, int b0)
{
    const int b = b0 + blockIdx.x;
    if (!D.active[b]) return;
    const BoxDev &X = D.box[b];
    const int l0 = X.centry, L = X.nlev;
    for (int i = l0; i < L - 1; ++i) {
        const BoxLev &V = X.lev[i], &C = X.lev[i + 1];
        const int n = V.n, m = C.n, M = m * m * m;
        double *phi = patch_phi(X, i, fid);
        const double inv_h2 = 1.0 / (V.h * V.h);
        for (int it = 0; it < nu1; ++it) cvp_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc);
        for (int q = threadIdx.x; q < M; q += CTPB) {
            const int I = q % m, J = (q / m) % m, K = q / (m * m);
            double sr = 0.0, sp = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int a = 2 * I + (c & 1), bb = 2 * J + ((c >> 1) & 1), dd = 2 * K + (c >> 2);
                const long r = lin(a, bb, dd, n);
                double Jd;
                sr += patch_op<KIND>(phi, a, bb, dd, n, inv_h2, load_c1<KIND>(V.coef, r), oc, Jd) - V.f[r];
                sp += phi[pidx(a, bb, dd, n)];
            }
            const double rp = sp / 8.0;
            C.phi[pidx(I, J, K, m)] = rp;
            C.phi0[q] = rp;
            C.tmp[q] = sr / 8.0;
        }
        __syncthreads();
        const double inv_H2 = 1.0 / (C.h * C.h);
        for (int q = threadIdx.x; q < M; q += CTPB) {
            const int I = q % m, J = (q / m) % m, K = q / (m * m);
            double Jd;
            C.f[q] = patch_op<KIND>(C.phi, I, J, K, m, inv_H2, load_c1<KIND>(C.coef, q), oc, Jd) - C.tmp[q];
        }
        __syncthreads();
    }
    {
        // coarsest level: its 32 sweeps from LDS when the padded iterate, the
        // source and the coefficient fit (every patch side of the usual
        // hierarchies ends at 3^3 to 10^3), else from global memory
        const BoxLev &V = X.lev[L - 1];
        double *phi = patch_phi(X, L - 1, fid);
        const double inv_h2 = 1.0 / (V.h * V.h);
        const int n = V.n, P = (n + 2) * (n + 2) * (n + 2), N = n * n * n;
        constexpr int NC = kNumCoef<KIND>();
        __shared__ double lds[kPatchCoarseLds];
        if (P + (1 + NC) * N <= kPatchCoarseLds) {
            double *sphi = lds, *sf = lds + P, *sc = lds + P + N;
            for (int q = threadIdx.x; q < P; q += CTPB) sphi[q] = phi[q];
            for (int q = threadIdx.x; q < N; q += CTPB) {
                sf[q] = V.f[q];
                if (NC >= 1) sc[q] = V.coef[q];
            }
            __syncthreads();
            for (int it = 0; it < kCoarseSweeps; ++it) cvp_sweep<KIND>(sphi, sf, sc, n, inv_h2, oc);
            for (int q = threadIdx.x; q < P; q += CTPB) phi[q] = sphi[q];
            __syncthreads();
        } else {
            for (int it = 0; it < kCoarseSweeps; ++it) cvp_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc);
        }
    }
    for (int i = L - 2; i >= l0; --i) {
        const BoxLev &V = X.lev[i], &C = X.lev[i + 1];
        const int n = V.n, m = C.n, N = n * n * n;
        double *phi = patch_phi(X, i, fid);
        const double inv_h2 = 1.0 / (V.h * V.h);
        for (int p = threadIdx.x; p < N; p += CTPB) {
            const int a = p % n, bb = (p / n) % n, dd = p / (n * n);
            const int I = a >> 1, J = bb >> 1, K = dd >> 1;
            const int Is[2] = {I, I + ((a & 1) ? 1 : -1)};
            const int Js[2] = {J, J + ((bb & 1) ? 1 : -1)};
            const int Ks[2] = {K, K + ((dd & 1) ? 1 : -1)};
            double v = 0.0;
            for (int c = 0; c < 8; ++c) {
                const int ox = c & 1, oy = (c >> 1) & 1, oz = c >> 2;
                const double w = (ox ? 0.25 : 0.75) * (oy ? 0.25 : 0.75) * (oz ? 0.25 : 0.75);
                double sign = 1.0;
                const int x = reflect_in(Is[ox], m, sign), y = reflect_in(Js[oy], m, sign),
                          z = reflect_in(Ks[oz], m, sign);
                v += w * (sign * (C.phi[pidx(x, y, z, m)] - C.phi0[lin(x, y, z, m)]));
            }
            phi[pidx(a, bb, dd, n)] += v;
        }
        __syncthreads();
        for (int it = 0; it < nu2; ++it) cvp_sweep<KIND>(phi, V.f, V.coef, n, inv_h2, oc);
    }
}

// ------------------------------------------------------------------- host

thread_local std::string b_err;

int bfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int bfail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b_err = buf;
    return code;
}

#define BHIP(expr)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return bfail(GR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)
#define BLAUNCH()                                                                                     \
    do {                                                                                              \
        hipError_t e_ = hipGetLastError();                                                            \
        if (e_ != hipSuccess) return bfail(GR_EDEVICE, "kernel launch: %s", hipGetErrorString(e_));   \
    } while (0)
#define BCHK(expr)                                                                                    \
    do {                                                                                              \
        int st_ = (expr);                                                                             \
        if (st_ != GR_OK) return st_;                                                                 \
    } while (0)

int num_levels(int n)
{
    int L = 1;
    while (n % 4 == 0) {
        n /= 2;
        ++L;
    }
    return L;
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

} // namespace

// prefix table of blocks per box for one launch shape
struct Tab {
    std::vector<int> start; // host copy
    int *dev = nullptr;
    int total() const { return start.back(); }
};

struct gr_batch_s {
    int nbox = 0;               // items: periodic boxes [0, nper), then patches [nper, nbox)
    int nper = 0, npatch = 0;
    gr_params prm{};
    int coarse_n = 16;
    std::vector<BoxDev> host;   // pointers into the workspace
    int maxdepth = 0;           // deepest multigrid level handled by grouped launches
    Tab fine;                   // fine level of every box
    Tab fine8;                  // the same, kSumPPT points per thread (sums, mean subtraction)
    std::vector<Tab> colour, cdom, coefr; // per depth
    std::vector<Tab> fz, fz64, fz16, colour_nf; // per depth: fused boxes (32x16, 64x16, 16x16 tiles), the others' colour passes
    // per depth and box: how level d is smoothed: 0 one launch per colour,
    // 1 fused 32x16, 2 fused 64x16, 3 fused 16x16, -1 not at all (only while tuning)
    std::vector<std::vector<signed char>> form;
    std::string tune_report;
    std::vector<Tab> rr;                        // per depth: residual + restriction (marching or per cell)
    Tab norms;                                  // stopping norms of the fine level
    bool use_march = true;
    bool use_fused = true;
    BatchDev D{};
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool use_graph = true;
    hipGraphExec_t graph[30]{};     // per field: the captured cycle (10 + field: patches, 20 + field: mixed)
    gr_solve_opts graph_opts[30]{}; // options it was captured with
    // patches: levels handled by grouped launches (depth < pmaxdepth), all levels (< pmaxlev)
    int pmaxdepth = 0, pmaxlev = 0;
    int pnest = 0; // deepest patch nesting (1: every patch's parent is a box)
    Tab pfine;                                  // interior cells of level 0
    // mixed precision (periodic boxes): grouped levels of the FP32 correction cycle
    int maxdepth32 = 0;
    std::vector<Tab> colour32, coarse32, rr32; // per depth: half cells, cells of the next level, residual + restriction
    std::vector<Tab> colour32nf;                  // per depth: half cells of the boxes not swept fused
    std::vector<Tab> pcell;                     // per level above a patch's entry: half its cells (colour passes)
    std::vector<Tab> pfz;                       // per level above a patch's entry: its 8^3 tiles (fused sweeps)
    bool pfused = true;                         // fused patch sweeps for even sweep counts (GRMG_PATCH_FUSED)
    int ptile = 0;                              // their tile: 0 = 8x8x8, 1 = 16x8x8, 2 = 16x16x8 (GRMG_PATCH_TILE)
    std::vector<Tab> pcellf;                    // per level above a patch's entry: its cells (prolongation)
    std::vector<Tab> pcoarse;                   // per depth d: interior cells of level d + 1 (grouped levels)
    std::vector<Tab> pcoefr;                    // per depth d: interior cells of level d + 1 (all levels)
    std::vector<Tab> pfaces;                    // per level: padded cells
    // patches run on their own stream and host thread, each field as soon as
    // the boxes' solve of that field is done (GRMG_BATCH_CONCURRENT=0: after
    // it on the batch's stream); own reduction scratch and activity flag
    BatchDev Dp{};
    double *p_partials = nullptr;
    int *p_any = nullptr;
    hipStream_t pstream = nullptr;
    hipEvent_t pdone = nullptr;
    bool conc = true;
    std::vector<double> rel_hist;   // [nbox][10] final relative residual per field
    std::vector<int> fb_hist;       // [nbox][10] mixed precision fell back to FP64 cycles
    double stall_ratio = 0.5;       // mixed precision: stalled refinement step ratio (GRMG_MIXED_STALL)
    double clock_khz = 0.0;
    long total_points = 0;
    // device task queue (GRMG_BATCH_QUEUE=1): levels of at most queue_n^3
    // points and the coarse cycle of every box in one persistent launch
    bool use_queue = false;
    int queue_n = 32;
    long queue_target = kQTarget;
    int qcap = 0;                   // task table capacity (nu1, nu2 <= kQueueMaxNu)
    QTask *qtasks = nullptr;        // device task table
    int *qctl = nullptr, *qdone = nullptr;
    int qcount = 0, qnu1 = -1, qnu2 = -1, qworkers = 0, cus = 0;
    std::vector<QTask> qhost;
};

namespace {

unsigned blocks_of(long items) { return (unsigned)((items + TPB - 1) / TPB); }

// workspace layout (base == nullptr: count only)
size_t batch_layout(gr_batch B, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    auto takeD = [&](size_t count) { return reinterpret_cast<double *>(take(sizeof(double) * count)); };
    for (int b = 0; b < B->nbox; ++b) {
        BoxDev &X = B->host[b];
        const long N = (long)X.lev[0].n * X.lev[0].n * X.lev[0].n;
        // iterate arrays of a patch carry a one-cell padding for the boundary values
        auto iter_len = [&](int n) { const long w = X.patch ? n + 2 : n; return w * w * w; };
        for (int f = 0; f < 10; ++f) X.field[f] = takeD(iter_len(X.lev[0].n));
        for (int s = 0; s < 5; ++s) X.src[s] = takeD(N);
        for (int c = 0; c < 6; ++c) X.A6[c] = takeD(N);
        X.AA = takeD(N);
        for (int c = 0; c < 3; ++c) X.fB[c] = takeD(N);
        for (int l = 0; l < X.nlev; ++l) {
            BoxLev &L = X.lev[l];
            const long M = (long)L.n * L.n * L.n;
            L.phi = l == 0 ? nullptr : takeD(iter_len(L.n));
            if (!X.patch) {
                auto takeF = [&](long count) { return reinterpret_cast<float *>(take(sizeof(float) * count)); };
                L.e = takeF(M);
                L.b32 = takeF(M);
                L.a32 = takeF(M);
                L.c32 = takeF(M);
                L.t32 = takeF(M);
            }
            L.phi0 = takeD(M);
            L.f = takeD(M);
            L.coef = takeD(M);
            L.tmp = takeD(M);
            L.ptmp = X.patch && l < X.centry ? takeD(iter_len(L.n)) : nullptr;
        }
    }
    auto takeI = [&](size_t count) { return reinterpret_cast<int *>(take(sizeof(int) * count)); };
    B->D.box = reinterpret_cast<const BoxDev *>(take(sizeof(BoxDev) * B->nbox));
    B->D.scal = takeD((size_t)B->nbox * B_NSCAL);
    B->D.active = takeI(B->nbox);
    B->D.cycles = takeI((size_t)B->nbox * 10);
    B->D.status = takeI(B->nbox);
    B->D.t_done = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * B->nbox * 10));
    B->D.t_start = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * 20));
    B->D.any_active = takeI(1);
    B->D.partials = takeD((size_t)B->fine.total() * 2 + 16);
    B->p_partials = takeD((size_t)B->pfine.total() * 2 + 16);
    B->p_any = takeI(1);
    B->qtasks = reinterpret_cast<QTask *>(take(sizeof(QTask) * (size_t)std::max(B->qcap, 1)));
    B->qctl = takeI(4);
    B->qdone = takeI(B->nbox);
    B->fine.dev = takeI(B->nbox + 1);
    B->fine8.dev = takeI(B->nbox + 1);
    B->norms.dev = takeI(B->nbox + 1);
    for (int d = 0; d < B->maxdepth; ++d) {
        B->colour[d].dev = takeI(B->nbox + 1);
        B->cdom[d].dev = takeI(B->nbox + 1);
        B->fz[d].dev = takeI(B->nbox + 1);
        B->fz64[d].dev = takeI(B->nbox + 1);
        B->fz16[d].dev = takeI(B->nbox + 1);
        B->rr[d].dev = takeI(B->nbox + 1);
        B->colour_nf[d].dev = takeI(B->nbox + 1);
    }
    for (size_t d = 0; d < B->coefr.size(); ++d) B->coefr[d].dev = takeI(B->nbox + 1);
    B->pfine.dev = takeI(B->nbox + 1);
    for (auto *v : {&B->pcell, &B->pfz, &B->pcellf, &B->pcoarse, &B->pcoefr, &B->pfaces, &B->colour32,
                    &B->coarse32, &B->rr32, &B->colour32nf})
        for (auto &T : *v) T.dev = takeI(B->nbox + 1);
    return off;
}

void make_tab(Tab &T, int nbox, const std::function<long(int)> &items)
{
    T.start.assign(nbox + 1, 0);
    for (int b = 0; b < nbox; ++b) T.start[b + 1] = T.start[b] + (int)blocks_of(items(b));
}

#define KDISPATCH(kind, KERNEL, GRID, BLOCK, ...)                                                      \
    do {                                                                                              \
        if ((kind) == GR_KIND_POISSON) KERNEL<GR_KIND_POISSON><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__);  \
        else if ((kind) == GR_KIND_HAMILTONIAN) KERNEL<GR_KIND_HAMILTONIAN><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); \
        else KERNEL<GR_KIND_CMC><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__);                                \
    } while (0)

OpConst opc(gr_batch B)
{
    OpConst o;
    o.kappa = 1.0 / (2.0 * B->prm.a * B->prm.a * B->prm.c_tilde * B->prm.c_tilde);
    o.A = 1.5 * B->prm.a * B->prm.omega_m;
    return o;
}

// The task table of the queue for V(nu1, nu2) cycles: per box, the phases of
// its levels from qentry down to the coarse cycle and back up, each split
// into z-ranges of about kQTarget points; emitted phase-major over the boxes,
// each task with the count of its box's tasks in earlier phases.
void q_build(const gr_batch B, int nu1, int nu2, std::vector<QTask> &out)
{
    out.clear();
    const auto &H = B->host;
    std::vector<std::vector<std::vector<QTask>>> ph(B->nper);
    for (int b = 0; b < B->nper; ++b) {
        const BoxDev &X = H[b];
        auto add = [&](int phase, int level, int planes, long plane_pts) {
            std::vector<QTask> v;
            const int pz = (int)std::max(1L, std::min((long)planes, (B->queue_target + plane_pts - 1) / plane_pts));
            for (int z0 = 0; z0 < planes; z0 += pz) v.push_back(QTask{b, phase, level, z0, std::min(planes, z0 + pz), 0});
            ph[b].push_back(v);
        };
        for (int i = X.qentry; i < X.centry; ++i) {
            const int n = X.lev[i].n, m = X.lev[i + 1].n;
            for (int it = 0; it < nu1; ++it) {
                add(Q_RED, i, n, (long)n * n / 2);
                add(Q_BLACK, i, n, (long)n * n / 2);
            }
            add(Q_RR, i, m, (long)m * m);
            add(Q_CRHS, i, m, (long)m * m);
        }
        add(Q_COARSE, X.centry, 1, 1);
        for (int i = X.centry - 1; i >= X.qentry; --i) {
            const int n = X.lev[i].n;
            add(Q_PROLONG, i, n, (long)n * n);
            for (int it = 0; it < nu2; ++it) {
                add(Q_RED, i, n, (long)n * n / 2);
                add(Q_BLACK, i, n, (long)n * n / 2);
            }
        }
    }
    size_t maxp = 0;
    for (const auto &v : ph) maxp = std::max(maxp, v.size());
    std::vector<int> prefix(B->nper, 0);
    for (size_t p = 0; p < maxp; ++p)
        for (int b = 0; b < B->nper; ++b) {
            if (p >= ph[b].size()) continue;
            for (QTask q : ph[b][p]) {
                q.prefix = prefix[b];
                out.push_back(q);
            }
            prefix[b] += (int)ph[b][p].size();
        }
}

// the task table for V(nu1, nu2) on the device (before any capture of a cycle)
int q_prepare(gr_batch B, int nu1, int nu2)
{
    if (!B->use_queue) return GR_OK;
    if (nu1 > kQueueMaxNu || nu2 > kQueueMaxNu)
        return bfail(GR_EINVAL, "the batch task queue takes nu1, nu2 <= %d", kQueueMaxNu);
    if (nu1 == B->qnu1 && nu2 == B->qnu2) return GR_OK;
    q_build(B, nu1, nu2, B->qhost);
    if ((int)B->qhost.size() > B->qcap) return bfail(GR_EDEVICE, "task table exceeds its capacity");
    BHIP(hipMemcpyAsync(B->qtasks, B->qhost.data(), sizeof(QTask) * B->qhost.size(), hipMemcpyHostToDevice, B->stream));
    BHIP(hipStreamSynchronize(B->stream));
    B->qcount = (int)B->qhost.size();
    B->qworkers = std::max(1, std::min(B->qcount, 2 * std::max(B->cus, 1)));
    B->qnu1 = nu1;
    B->qnu2 = nu2;
    return GR_OK;
}

// pin (all boxes or active ones): mean then subtract
int batch_pin(gr_batch B, int fid, int active_only)
{
    hipStream_t s = B->stream;
    kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 0, opc(B), active_only);
    kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_MEAN, -1, active_only, 0);
    kb_sub_mean<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, active_only);
    BLAUNCH();
    return GR_OK;
}

// one cycle of the batch: frozen means, norms, control, V-cycle, pin
// nu sweeps of level d of every box: fused (out of place, an even count ends
// in phi) for the boxes that take 32x16 tiles, one launch per colour for the rest
template <int TX, int TY>
void launch_kb_fused(hipStream_t s, int kind, const Tab &T, BatchDev D, int d, int fid, int it, OpConst oc)
{
    constexpr int NT = (TX / 2) * TY;
    if (kind == GR_KIND_POISSON) kb_fused<GR_KIND_POISSON, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, fid, it, oc);
    else if (kind == GR_KIND_HAMILTONIAN)
        kb_fused<GR_KIND_HAMILTONIAN, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, fid, it, oc);
    else kb_fused<GR_KIND_CMC, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, fid, it, oc);
}

void batch_smooth(gr_batch B, int kind, int d, int fid, int nu)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    // the fused forms work out of place in pairs of sweeps
    const bool fused = nu % 2 == 0 && (B->fz[d].total() > 0 || B->fz64[d].total() > 0 || B->fz16[d].total() > 0);
    const Tab &TC = fused ? B->colour_nf[d] : B->colour[d];
    for (int it = 0; it < nu; ++it) {
        if (fused && B->fz[d].total()) launch_kb_fused<32, 16>(s, kind, B->fz[d], B->D, d, fid, it, oc);
        if (fused && B->fz64[d].total()) launch_kb_fused<64, 16>(s, kind, B->fz64[d], B->D, d, fid, it, oc);
        if (fused && B->fz16[d].total()) launch_kb_fused<16, 16>(s, kind, B->fz16[d], B->D, d, fid, it, oc);
        if (TC.total() > 0)
            for (int colour = 0; colour < 2; ++colour)
                KDISPATCH(kind, kb_colour, TC.total(), TPB, B->D, TC.dev, d, fid, colour, oc);
    }
}

// FP32 correction smoothing at depth d: boxes whose level d is swept fused
// (forms 1, 2: the FP64 tables fz / fz64) and the rest one launch per colour
void smooth32_tab(gr_batch B, int d)
{
    const auto &H = B->host;
    make_tab(B->colour32nf[d], B->nbox, [&](int b) {
        if (H[b].patch || d >= H[b].centry32) return 0L;
        const bool fused = d < (int)B->form.size() && B->form[d][b] >= 1;
        const long n = H[b].lev[d].n;
        return fused ? 0L : n * n * n / 2;
    });
}

// smoothing tables of depth d from the boxes' forms
void smooth_tabs(gr_batch B, int d)
{
    const auto &H = B->host;
    const auto &F = B->form[d];
    const int nb = B->nbox;
    auto blocks = [&](int b, int tx, int ty) { const long n = H[b].lev[d].n; return (n / tx) * (n / ty) * (n / kFZ); };
    // block counts for the 512-thread 64x16 launches, as items of TPB threads
    make_tab(B->fz[d], nb, [&](int b) { return F[b] == 1 ? blocks(b, 32, 16) * TPB : 0L; });
    make_tab(B->fz64[d], nb, [&](int b) { return F[b] == 2 ? blocks(b, 64, 16) * TPB : 0L; });
    make_tab(B->fz16[d], nb, [&](int b) { return F[b] == 3 ? blocks(b, 16, 16) * TPB : 0L; });
    make_tab(B->colour_nf[d], nb, [&](int b) { long n = H[b].lev[d].n; return F[b] == 0 ? n * n * n / 2 : 0L; });
    if (d < (int)B->colour32nf.size()) smooth32_tab(B, d);
}

int batch_cycle(gr_batch B, int kind, int fid, const gr_solve_opts &o)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    if (kind == GR_KIND_HAMILTONIAN) {
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 1, oc, 1);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FBAR, -1, 1, 0);
    } else if (kind == GR_KIND_CMC) {
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 2, oc, 1);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FSHIFT, B_FMEAN, 1, 0);
    }
    KDISPATCH(kind, kb_norms_m, B->norms.total(), TPB, B->D, B->norms.dev, fid, oc);
    kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->norms.dev, 2, B_RN, -1, 1, 0);
    kb_control<<<1, 1024, 0, s>>>(B->D, fid, o.rtol, o.max_cycles, 0, B->nper, -1.0);
    // descent through the levels handled by grouped launches
    for (int d = 0; d < B->maxdepth; ++d) {
        const Tab &TC = B->colour[d], &TD = B->cdom[d];
        if (TC.total() == 0) continue;
        batch_smooth(B, kind, d, fid, o.nu1);
        KDISPATCH(kind, kb_rr_m, B->rr[d].total(), TPB, B->D, B->rr[d].dev, d, fid, oc);
        KDISPATCH(kind, kb_coarse_rhs, TD.total(), TPB, B->D, TD.dev, d, oc);
    }
    if (B->use_queue) { // the levels from each box's queue entry and its coarse cycle: one persistent launch
        kb_queue_reset<<<1, 1024, 0, s>>>(B->qctl, B->qdone, B->nbox, 0);
        KDISPATCH(kind, kb_queue, B->qworkers, CTPB, B->D, B->qtasks, B->qcount, B->qctl, B->qdone, fid, o.nu1, o.nu2,
                  oc, kQSpin);
    } else {
        KDISPATCH(kind, kb_coarse_vcycle, B->nper, CTPB, B->D, fid, o.nu1, o.nu2, oc);
    }
    for (int d = B->maxdepth - 1; d >= 0; --d) {
        const Tab &TC = B->colour[d], &TD = B->cdom[d];
        if (TC.total() == 0) continue;
        kb_coarse_diff<<<TD.total(), TPB, 0, s>>>(B->D, TD.dev, d);
        kb_prolong_cell<<<TD.total(), TPB, 0, s>>>(B->D, TD.dev, d, fid);
        batch_smooth(B, kind, d, fid, o.nu2);
        (void)TD;
    }
    // the Poisson cycle commutes with adding a constant: those fields are pinned
    // once after the loop (batch_field), the nonlinear kinds after every cycle
    if (kind != GR_KIND_POISSON) BCHK(batch_pin(B, fid, 1));
    BLAUNCH();
    return GR_OK;
}

} // namespace

namespace {

// Replays (or captures, then replays) one cycle of items [b0, b1) until the
// device control reports no active item; graph slot `slot`.  Then reads the
// final relative residuals of those items for field fid.
template <class Body>
int run_cycles(gr_batch B, hipStream_t s, const int *any_dev, int slot, const gr_solve_opts &o, Body cycle)
{
    const bool graph = B->use_graph && s != nullptr;
    hipGraphExec_t &ge = B->graph[slot];
    const gr_solve_opts &go = B->graph_opts[slot];
    if (ge && (go.nu1 != o.nu1 || go.nu2 != o.nu2 || go.max_cycles != o.max_cycles || go.rtol != o.rtol)) {
        (void)hipGraphExecDestroy(ge);
        ge = nullptr;
    }
    for (int it = 0;; ++it) {
        if (graph) {
            if (!ge) {
                hipGraph_t gr;
                BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                int st = cycle();
                hipError_t e = hipStreamEndCapture(s, &gr);
                if (st != GR_OK) return st;
                if (e != hipSuccess) return bfail(GR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
                e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e != hipSuccess) return bfail(GR_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
                B->graph_opts[slot] = o;
            }
            BHIP(hipGraphLaunch(ge, s));
        } else {
            BCHK(cycle());
        }
        int any = 0;
        BHIP(hipMemcpyAsync(&any, any_dev, sizeof any, hipMemcpyDeviceToHost, s));
        BHIP(hipStreamSynchronize(s));
        if (!any) break;
        if (it > o.max_cycles + 2) return bfail(GR_EDEVICE, "batch control did not stop");
    }
    return GR_OK;
}

int read_rel(gr_batch B, hipStream_t s, int fid, int b0, int b1)
{
    std::vector<double> sc((size_t)B->nbox * B_NSCAL);
    BHIP(hipMemcpyAsync(sc.data(), B->D.scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    for (int b = b0; b < b1; ++b) {
        B->rel_hist[(size_t)b * 10 + fid] = sc[(size_t)b * B_NSCAL + B_REL];
        B->fb_hist[(size_t)b * 10 + fid] = sc[(size_t)b * B_NSCAL + B_FB] != 0.0;
    }
    return GR_OK;
}

int batch_field(gr_batch B, int kind, int fid, const gr_solve_opts &o)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    kb_begin_field<<<1, 1024, 0, s>>>(B->D, fid, 0, B->nper, fid);
    if (kind != GR_KIND_POISSON)
        for (size_t d = 0; d < B->coefr.size(); ++d)
            if (B->coefr[d].total())
                kb_restrict_coef<<<B->coefr[d].total(), TPB, 0, s>>>(B->D, B->coefr[d].dev, (int)d);
    if (kind == GR_KIND_CMC) {
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 3, oc, 0);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FMEAN, -1, 0, 0);
    }
    BLAUNCH();
    BCHK(q_prepare(B, o.nu1, o.nu2));
    BCHK(batch_pin(B, fid, 0));
    BCHK(run_cycles(B, s, B->D.any_active, fid, o, [&] { return batch_cycle(B, kind, fid, o); }));
    if (kind == GR_KIND_POISSON) BCHK(batch_pin(B, fid, 0));
    return read_rel(B, s, fid, 0, B->nper);
}

#define LDISPATCH(kind, KERNEL, GRID, BLOCK, ...)                                                      \
    do {                                                                                              \
        if ((kind) == GR_KIND_POISSON) KERNEL<K_LIN_POISSON><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__);    \
        else if ((kind) == GR_KIND_HAMILTONIAN) KERNEL<K_LIN_HAM><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__); \
        else KERNEL<K_LIN_CMC><<<GRID, BLOCK, 0, s>>>(__VA_ARGS__);                                  \
    } while (0)

template <int TX, int TY>
void launch_kb32_fused(hipStream_t s, int kind, const Tab &T, BatchDev D, int d, int it, OpConst oc)
{
    constexpr int NT = (TX / 2) * TY;
    if (kind == GR_KIND_POISSON) kb32_fused<K_LIN_POISSON, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, it, oc);
    else if (kind == GR_KIND_HAMILTONIAN) kb32_fused<K_LIN_HAM, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, it, oc);
    else kb32_fused<K_LIN_CMC, TX, TY><<<T.total(), NT, 0, s>>>(D, T.dev, d, it, oc);
}

// nu sweeps of the correction on level d of every box: fused where the box's
// form says so (an even count ends in e), one launch per colour elsewhere
void batch_smooth32(gr_batch B, int kind, int d, int nu)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    const bool formed = d < B->maxdepth;
    const bool fused =
        formed && nu % 2 == 0 && (B->fz[d].total() > 0 || B->fz64[d].total() > 0 || B->fz16[d].total() > 0);
    const Tab &TC = fused ? B->colour32nf[d] : B->colour32[d];
    for (int it = 0; it < nu; ++it) {
        if (fused && B->fz[d].total()) launch_kb32_fused<32, 16>(s, kind, B->fz[d], B->D, d, it, oc);
        if (fused && B->fz64[d].total()) launch_kb32_fused<64, 16>(s, kind, B->fz64[d], B->D, d, it, oc);
        if (fused && B->fz16[d].total()) launch_kb32_fused<16, 16>(s, kind, B->fz16[d], B->D, d, it, oc);
        if (TC.total() > 0)
            for (int colour = 0; colour < 2; ++colour)
                LDISPATCH(kind, kb32_colour, TC.total(), TPB, B->D, TC.dev, d, colour, oc);
    }
}

// one refinement step of every active box: frozen means, FP64 residual and
// stopping test, FP32 correction V-cycle, FP64 update
int batch_cycle_mixed(gr_batch B, int kind, int fid, const gr_solve_opts &o)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    if (kind == GR_KIND_HAMILTONIAN) {
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 1, oc, 1);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FBAR, -1, 1, 0);
    } else if (kind == GR_KIND_CMC) {
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 2, oc, 1);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FSHIFT, B_FMEAN, 1, 0);
    }
    KDISPATCH(kind, kb_ir_m, B->norms.total(), TPB, B->D, B->norms.dev, fid, oc);
    kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->norms.dev, 2, B_RN, -1, 1, 0);
    kb_control<<<1, 1024, 0, s>>>(B->D, fid, o.rtol, o.max_cycles, 0, B->nper, B->stall_ratio);
    if (kind == GR_KIND_HAMILTONIAN) // the linearisation frozen at this iterate, on every level
        for (size_t d = 0; d < B->coefr.size(); ++d)
            if (B->coefr[d].total())
                for (int which = 0; which < 2; ++which)
                    kb_restrict32<<<B->coefr[d].total(), TPB, 0, s>>>(B->D, B->coefr[d].dev, (int)d, which);
    kb32_fill<<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, 0); // the correction starts from e = 0
    for (int d = 0; d < B->maxdepth32; ++d) {
        if (B->colour32[d].total() == 0) continue;
        batch_smooth32(B, kind, d, o.nu1);
        LDISPATCH(kind, kb32_lin_rr, B->rr32[d].total(), TPB, B->D, B->rr32[d].dev, d, oc);
    }
    LDISPATCH(kind, kb32_coarse, B->nper, kCoarseThreads, B->D, o.nu1, o.nu2, oc);
    for (int d = B->maxdepth32 - 1; d >= 0; --d) {
        const Tab &TC = B->colour32[d];
        if (TC.total() == 0) continue;
        kb32_prolong<<<B->coarse32[d].total(), TPB, 0, s>>>(B->D, B->coarse32[d].dev, d);
        batch_smooth32(B, kind, d, o.nu2);
    }
    kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 7, oc, 1);
    kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_MEAN, -1, 1, 0);
    kb_ir_update<<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid);
    BLAUNCH();
    return GR_OK;
}

int batch_field_mixed(gr_batch B, int kind, int fid, const gr_solve_opts &o)
{
    hipStream_t s = B->stream;
    const OpConst oc = opc(B);
    kb_begin_field<<<1, 1024, 0, s>>>(B->D, fid, 0, B->nper, fid);
    if (kind == GR_KIND_CMC) { // <f>, and c = -m2 in FP32 on every level (fixed for the solve)
        kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, fid, 3, oc, 0);
        kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_FMEAN, -1, 0, 0);
        kb_neg_coef32<<<B->fine.total(), TPB, 0, s>>>(B->D, B->fine.dev);
        for (size_t d = 0; d < B->coefr.size(); ++d)
            if (B->coefr[d].total())
                kb_restrict32<<<B->coefr[d].total(), TPB, 0, s>>>(B->D, B->coefr[d].dev, (int)d, 0);
    }
    BLAUNCH();
    BCHK(batch_pin(B, fid, 0));
    BCHK(run_cycles(B, s, B->D.any_active, 20 + fid, o, [&] { return batch_cycle_mixed(B, kind, fid, o); }));
    // items whose refinement stalled finish with FP64 FAS cycles from their
    // current iterate, the cycle count continuing
    kb_activate_fallback<<<1, 1024, 0, s>>>(B->D, 0, B->nper, 1);
    BLAUNCH();
    int any = 0;
    BHIP(hipMemcpyAsync(&any, B->D.any_active, sizeof any, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (any) {
        if (kind != GR_KIND_POISSON)
            for (size_t d = 0; d < B->coefr.size(); ++d)
                if (B->coefr[d].total())
                    kb_restrict_coef<<<B->coefr[d].total(), TPB, 0, s>>>(B->D, B->coefr[d].dev, (int)d);
        BLAUNCH();
        BCHK(q_prepare(B, o.nu1, o.nu2));
        BCHK(run_cycles(B, s, B->D.any_active, fid, o, [&] { return batch_cycle(B, kind, fid, o); }));
        if (kind == GR_KIND_POISSON) { // the FP64 cycles pin once at the end
            kb_activate_fallback<<<1, 1024, 0, s>>>(B->D, 0, B->nper, 1);
            BCHK(batch_pin(B, fid, 1));
            kb_activate_fallback<<<1, 1024, 0, s>>>(B->D, 0, B->nper, 0);
            BLAUNCH();
        }
    }
    return read_rel(B, s, fid, 0, B->nper);
}

// ------------------------------------------------------------ patch cycle

#define PFUSED(kind, TX, TY, TZ)                                                                      \
    do {                                                                                              \
        if ((kind) == GR_KIND_POISSON)                                                                \
            kp_fused<GR_KIND_POISSON, TX, TY, TZ><<<grid8, TPB, 0, s>>>(B->Dp, T.dev, d, fid, it, oc);  \
        else if ((kind) == GR_KIND_HAMILTONIAN)                                                       \
            kp_fused<GR_KIND_HAMILTONIAN, TX, TY, TZ><<<grid8, TPB, 0, s>>>(B->Dp, T.dev, d, fid, it, oc); \
        else                                                                                          \
            kp_fused<GR_KIND_CMC, TX, TY, TZ><<<grid8, TPB, 0, s>>>(B->Dp, T.dev, d, fid, it, oc); \
    } while (0)

void patch_smooth(gr_batch B, hipStream_t s, int kind, int d, int fid, int nu)
{
    const OpConst oc = opc(B);
    if (B->pfused && nu % 2 == 0) { // an even count of out-of-place sweeps ends in the iterate
        const Tab &T = B->pfz[d];
        const unsigned grid8 = (unsigned)((T.total() + 7) / 8 * 8);
        for (int it = 0; it < nu; ++it) {
            if (B->ptile == 2) PFUSED(kind, 16, 16, 8);
            else if (B->ptile == 1) PFUSED(kind, 16, 8, 8);
            else PFUSED(kind, 8, 8, 8);
        }
        return;
    }
    const Tab &T = B->pcell[d];
    for (int it = 0; it < nu; ++it)
        for (int colour = 0; colour < 2; ++colour)
            KDISPATCH(kind, kp_colour, T.total(), TPB, B->Dp, T.dev, d, fid, colour, oc);
}

// one cycle of every patch: norms, control, V-cycle (no pin, no frozen means)
int patch_cycle(gr_batch B, hipStream_t s, int kind, int fid, const gr_solve_opts &o)
{
    const OpConst oc = opc(B);
    KDISPATCH(kind, kp_norms, B->pfine.total(), TPB, B->Dp, B->pfine.dev, fid, oc);
    kb_finalize<<<B->npatch, TPB, 0, s>>>(B->Dp, B->pfine.dev, 2, B_RN, -1, 1, B->nper);
    kb_control<<<1, 1024, 0, s>>>(B->Dp, fid, o.rtol, o.max_cycles, B->nper, B->nbox, -1.0);
    for (int d = 0; d < B->pmaxdepth; ++d) {
        if (B->pcell[d].total() == 0) continue;
        patch_smooth(B, s, kind, d, fid, o.nu1);
        const Tab &TC = B->pcoarse[d];
        KDISPATCH(kind, kp_rr, TC.total(), TPB, B->Dp, TC.dev, d, fid, oc);
        KDISPATCH(kind, kp_coarse_rhs, TC.total(), TPB, B->Dp, TC.dev, d, oc);
    }
    KDISPATCH(kind, kp_coarse_vcycle, B->npatch, CTPB, B->Dp, fid, o.nu1, o.nu2, oc, B->nper);
    for (int d = B->pmaxdepth - 1; d >= 0; --d) {
        if (B->pcell[d].total() == 0) continue;
        kp_prolong<<<B->pcellf[d].total(), TPB, 0, s>>>(B->Dp, B->pcellf[d].dev, d, fid);
        patch_smooth(B, s, kind, d, fid, o.nu2);
    }
    BLAUNCH();
    return GR_OK;
}

// boundary values of every level of every patch from the parents' field fid
void patch_faces(gr_batch B, hipStream_t s, int fid)
{
    for (int l = 0; l < B->pmaxlev; ++l)
        if (B->pfaces[l].total()) kp_faces<<<B->pfaces[l].total(), TPB, 0, s>>>(B->Dp, B->pfaces[l].dev, l, fid);
}

// field fid of every patch, nesting depth by depth: each depth's boundary
// values come from the finished field of the depth above (reading D6)
int patch_field(gr_batch B, hipStream_t s, int kind, int fid, const gr_solve_opts &o)
{
    kb_begin_field<<<1, 1024, 0, s>>>(B->Dp, fid, B->nper, B->nbox, 10 + fid);
    if (kind != GR_KIND_POISSON)
        for (size_t d = 0; d < B->pcoefr.size(); ++d)
            if (B->pcoefr[d].total())
                kp_restrict_coef<<<B->pcoefr[d].total(), TPB, 0, s>>>(B->Dp, B->pcoefr[d].dev, (int)d);
    for (int depth = 1; depth <= B->pnest; ++depth) {
        if (B->pnest > 1) kb_activate_depth<<<1, 1024, 0, s>>>(B->Dp, B->nper, B->nbox, depth);
        patch_faces(B, s, fid);
        BLAUNCH();
        BCHK(run_cycles(B, s, B->Dp.any_active, 10 + fid, o, [&] { return patch_cycle(B, s, kind, fid, o); }));
    }
    return read_rel(B, s, fid, B->nper, B->nbox);
}

} // namespace

extern "C" {

const char *gr_batch_last_error(void) { return b_err.c_str(); }

} // extern "C"

namespace {

// Levels of a patch: halve while n is even and n/2 >= 3.
int patch_levels(int n)
{
    int L = 1;
    while (n % 2 == 0 && n / 2 >= 3) {
        n /= 2;
        ++L;
    }
    return L;
}

constexpr int kPatchCoarseN = 16; // patch levels at or below this size: single-workgroup cycle

int create_batch(const gr_grid_desc *descs, int count, const gr_patch_desc *patches, int npatch,
                 const gr_params *prm, gr_batch *out)
{
    if (!descs || !prm || !out || (npatch > 0 && !patches)) return bfail(GR_EINVAL, "null argument");
    *out = nullptr;
    if (count < 1 || npatch < 0 || count + npatch > kMaxBoxes)
        return bfail(GR_EINVAL, "%d boxes + %d patches outside 1..%d items", count, npatch, kMaxBoxes);
    if (!(prm->a > 0.0) || !(prm->c_tilde > 0.0) || !std::isfinite(prm->omega_m))
        return bfail(GR_EINVAL, "a and c_tilde must be positive");
    for (int j = 0; j < npatch; ++j) {
        const gr_patch_desc &q = patches[j];
        const bool origin_ok = std::fabs(q.origin[0]) <= 1e6 && std::fabs(q.origin[1]) <= 1e6 &&
                               std::fabs(q.origin[2]) <= 1e6; // false for NaN
        if (q.n < 3 || q.n > 512 || !(q.h > 0.0) || !(q.h <= 1e3) || q.parent < 0 || q.parent >= count + j ||
            !origin_ok)
            return bfail(GR_EINVAL,
                         "patch %d: n = %d must be 3..512, 0 < h <= 1e3, parent a box or an earlier patch, "
                         "|origin| <= 1e6",
                         j, q.n);
        if (q.parent >= count) { // nested: every sample strictly between the parent patch's cell centres
            const gr_patch_desc &P = patches[q.parent - count];
            for (int a = 0; a < 3; ++a) {
                const double glo = (q.origin[a] - 0.5 * q.h) / P.h - 0.5;
                const double ghi = (q.origin[a] + (q.n + 0.5) * q.h) / P.h - 0.5;
                if (!(glo > 0.0) || !(ghi < P.n - 1.0))
                    return bfail(GR_EINVAL, "patch %d: must lie at least (H + h)/2 inside its parent patch %d",
                                 j, q.parent - count);
            }
        }
    }
    gr_batch B = new (std::nothrow) gr_batch_s();
    if (!B) return bfail(GR_EINVAL, "out of host memory");
    B->nbox = count + npatch;
    B->nper = count;
    B->npatch = npatch;
    B->prm = *prm;
    if (const char *e = std::getenv("GRMG_COARSE_N")) B->coarse_n = std::max(2, std::atoi(e));
    if (const char *e = std::getenv("GRMG_MIXED_STALL")) B->stall_ratio = std::atof(e);
    if (const char *e = std::getenv("GRMG_BATCH_QUEUE")) B->use_queue = std::atoi(e) != 0;
    if (const char *e = std::getenv("GRMG_PATCH_FUSED")) B->pfused = std::atoi(e) != 0;
    if (const char *e = std::getenv("GRMG_PATCH_TILE")) B->ptile = std::min(2, std::max(0, std::atoi(e)));
    if (const char *e = std::getenv("GRMG_QUEUE_N")) B->queue_n = std::max(2, std::atoi(e));
    if (const char *e = std::getenv("GRMG_QUEUE_TARGET")) B->queue_target = std::max(64L, std::atol(e));
    if (const char *e = std::getenv("GRMG_BATCH_GRAPH")) B->use_graph = std::atoi(e) != 0;
    if (const char *e = std::getenv("GRMG_BATCH_CONCURRENT")) B->conc = std::atoi(e) != 0;
    B->host.resize(count + npatch);
    int maxd = 0, maxc = 0;
    for (int b = 0; b < count; ++b) {
        const int n = descs[b].n;
        if (n < 2 || (n & 1) || n > 1024 || !(descs[b].h > 0.0)) {
            delete B;
            return bfail(GR_EINVAL, "item %d: n = %d must be even, 2..1024, h > 0", b, n);
        }
        BoxDev &X = B->host[b];
        std::memset(&X, 0, sizeof X);
        X.nlev = num_levels(n);
        X.centry = X.nlev - 1;
        for (int l = 0; l < X.nlev; ++l) {
            X.lev[l].n = n >> l;
            X.lev[l].h = descs[b].h * (double)(1 << l);
            if ((n >> l) <= B->coarse_n && X.centry == X.nlev - 1 && l < X.centry) X.centry = l;
        }
        X.qentry = X.centry;
        if (B->use_queue)
            for (int l = 0; l < X.centry; ++l)
                if (X.lev[l].n <= B->queue_n) {
                    X.qentry = l;
                    break;
                }
        X.centry32 = X.nlev - 1; // FP32 correction cycle: single workgroup from 8^3 down
        for (int l = 0; l < X.nlev - 1; ++l)
            if (X.lev[l].n <= 8) {
                X.centry32 = l;
                break;
            }
        B->maxdepth32 = std::max(B->maxdepth32, X.centry32);
        maxd = std::max(maxd, X.centry);
        maxc = std::max(maxc, X.nlev - 1);
        B->total_points += (long)n * n * n;
    }
    B->maxdepth = maxd;
    int pmaxd = 0, pmaxl = 0;
    for (int j = 0; j < npatch; ++j) {
        const gr_patch_desc &q = patches[j];
        BoxDev &X = B->host[count + j];
        std::memset(&X, 0, sizeof X);
        X.patch = 1;
        X.parent = q.parent;
        X.depth = q.parent < count ? 1 : B->host[q.parent].depth + 1;
        B->pnest = std::max(B->pnest, X.depth);
        for (int a = 0; a < 3; ++a) X.origin[a] = q.origin[a];
        X.nlev = patch_levels(q.n);
        X.centry = X.nlev - 1;
        for (int l = 0; l < X.nlev; ++l) {
            X.lev[l].n = q.n >> l;
            X.lev[l].h = q.h * (double)(1 << l);
            if ((q.n >> l) <= kPatchCoarseN && X.centry == X.nlev - 1 && l < X.centry) X.centry = l;
        }
        X.qentry = X.centry;
        pmaxd = std::max(pmaxd, X.centry);
        pmaxl = std::max(pmaxl, X.nlev);
        B->total_points += (long)q.n * q.n * q.n;
    }
    B->pmaxdepth = pmaxd;
    B->pmaxlev = pmaxl;
    const int nb = count + npatch;
    auto &H = B->host;
    // periodic tables: no blocks for patches
    make_tab(B->fine, nb, [&](int b) { long n = H[b].patch ? 0 : H[b].lev[0].n; return n * n * n; });
    make_tab(B->fine8, nb, [&](int b) {
        long n = H[b].patch ? 0 : H[b].lev[0].n;
        return (n * n * n + kSumPPT - 1) / kSumPPT;
    });
    B->colour.resize(maxd);
    B->cdom.resize(maxd);
    B->fz.resize(maxd);
    B->fz64.resize(maxd);
    B->fz16.resize(maxd);
    B->rr.resize(maxd);
    if (const char *e = std::getenv("GRMG_MARCH")) B->use_march = std::atoi(e) != 0;
    B->D.march = B->use_march ? 1 : 0;
    make_tab(B->norms, nb, [&](int b) {
        if (H[b].patch) return 0L;
        const long n = H[b].lev[0].n;
        return B->use_march && marchable((int)n) ? march_blocks((int)n) * TPB : n * n * n;
    });
    B->colour_nf.resize(maxd);
    if (const char *e = std::getenv("GRMG_BATCH_FUSED")) B->use_fused = std::atoi(e) != 0;
    auto fusable = [&](int b, int d) {
        const int n = H[b].lev[d].n;
        return !H[b].patch && d < H[b].qentry && n >= 64 && n % 32 == 0;
    };
    // levels of periodic boxes run by grouped launches: above the queue entry
    // (the coarse cycle's entry when the queue is off)
    auto grouped = [&](int b, int d) { return !H[b].patch && d < H[b].qentry; };
    for (int d = 0; d < maxd; ++d) {
        make_tab(B->colour[d], nb, [&](int b) { long n = H[b].lev[d].n; return grouped(b, d) ? n * n * n / 2 : 0L; });

        make_tab(B->rr[d], nb, [&](int b) {
            if (!grouped(b, d)) return 0L;
            const long n = H[b].lev[d].n, m = H[b].lev[d + 1].n;
            return B->use_march && marchable((int)n) ? march_blocks((int)n) * TPB : m * m * m;
        });

        make_tab(B->cdom[d], nb, [&](int b) { long m = grouped(b, d) ? H[b].lev[d + 1].n : 0; return m * m * m; });
    }
    // untuned forms: 32x16 fused sweeps where they tile, else one launch per colour
    // GRMG_BATCH_FORM = 3: the 16x16 fused form wherever the 32x16 one does not
    // apply and the side allows it (a test knob; the autotuner chooses otherwise)
    int extra16 = 0;
    if (const char *e = std::getenv("GRMG_BATCH_FORM")) extra16 = std::atoi(e) == 3;
    B->form.assign(maxd, std::vector<signed char>(nb, 0));
    for (int d = 0; d < maxd; ++d) {
        for (int b = 0; b < nb; ++b) {
            const int n = H[b].lev[d].n;
            B->form[d][b] = !grouped(b, d) ? -1
                            : !B->use_fused ? 0
                            : fusable(b, d) ? 1
                            : (extra16 && n >= 32 && n % 16 == 0) ? 3 : 0;
        }
        smooth_tabs(B, d);
    }
    B->coefr.resize(maxc);
    for (int d = 0; d < maxc; ++d)
        make_tab(B->coefr[d], nb, [&](int b) {
            long m = !H[b].patch && d + 1 < H[b].nlev ? H[b].lev[d + 1].n : 0;
            return m * m * m;
        });
    // FP32 correction cycle tables (periodic boxes, levels above their FP32 entry)
    B->colour32.resize(B->maxdepth32);
    B->coarse32.resize(B->maxdepth32);
    B->rr32.resize(B->maxdepth32);
    B->colour32nf.resize(B->maxdepth32);
    for (int d = 0; d < B->maxdepth32; ++d) {
        auto on = [&](int b) { return !H[b].patch && d < H[b].centry32; };
        make_tab(B->colour32[d], nb, [&](int b) { long n = on(b) ? H[b].lev[d].n : 0; return n * n * n / 2; });
        make_tab(B->coarse32[d], nb, [&](int b) { long m = on(b) ? H[b].lev[d + 1].n : 0; return m * m * m; });
        make_tab(B->rr32[d], nb, [&](int b) {
            if (!on(b)) return 0L;
            const long n = H[b].lev[d].n, m = H[b].lev[d + 1].n;
            return B->use_march && marchable((int)n) ? march_blocks((int)n) * TPB : m * m * m;
        });
        smooth32_tab(B, d); // after the forms (built above)
    }
    // patch tables: no blocks for periodic boxes
    auto cells = [&](int b, int l) { long n = H[b].patch && l < H[b].nlev ? H[b].lev[l].n : 0; return n * n * n; };
    make_tab(B->pfine, nb, [&](int b) { return cells(b, 0); });
    B->pcell.resize(pmaxd);
    B->pfz.resize(pmaxd);
    B->pcellf.resize(pmaxd);
    B->pcoarse.resize(pmaxd);
    for (int d = 0; d < pmaxd; ++d) {
        // levels above the entry have n > 16 and even n (they were halved)
        make_tab(B->pcell[d], nb, [&](int b) { return d < H[b].centry ? cells(b, d) / 2 : 0L; });
        make_tab(B->pfz[d], nb, [&](int b) {
            if (!(H[b].patch && d < H[b].centry)) return 0L;
            const long n = H[b].lev[d].n, tx = B->ptile >= 1 ? 16 : 8, ty = B->ptile >= 2 ? 16 : 8;
            return ((n + tx - 1) / tx) * ((n + ty - 1) / ty) * ((n + 7) / 8) * TPB;
        });
        make_tab(B->pcellf[d], nb, [&](int b) { return d < H[b].centry ? cells(b, d) : 0L; });
        make_tab(B->pcoarse[d], nb, [&](int b) { return d < H[b].centry ? cells(b, d + 1) : 0L; });
    }
    B->pcoefr.resize(std::max(pmaxl - 1, 0));
    for (int d = 0; d + 1 < pmaxl; ++d) make_tab(B->pcoefr[d], nb, [&](int b) { return cells(b, d + 1); });
    B->pfaces.resize(pmaxl);
    for (int l = 0; l < pmaxl; ++l)
        make_tab(B->pfaces[l], nb, [&](int b) {
            long w = H[b].patch && l < H[b].nlev ? H[b].lev[l].n + 2 : 0;
            return w * w * w;
        });
    if (B->use_queue) {
        std::vector<QTask> t;
        q_build(B, kQueueMaxNu, kQueueMaxNu, t);
        B->qcap = (int)t.size();
    }
    B->ws_bytes = batch_layout(B, nullptr);
    *out = B;
    return GR_OK;
}

} // namespace

extern "C" {

int gr_create_batch(const gr_grid_desc *descs, int count, const gr_params *prm, gr_batch *out)
{
    return create_batch(descs, count, nullptr, 0, prm, out);
}

int gr_create_batch_patches(const gr_grid_desc *boxes, int nbox, const gr_patch_desc *patches, int npatch,
                            const gr_params *prm, gr_batch *out)
{
    return create_batch(boxes, nbox, patches, npatch, prm, out);
}

int gr_batch_workspace_bytes(gr_batch B, size_t *bytes)
{
    if (!B || !bytes) return bfail(GR_EINVAL, "null argument");
    *bytes = B->ws_bytes;
    return GR_OK;
}

int gr_batch_bind(gr_batch B, void *d_ws, size_t bytes, void *stream)
{
    if (!B || !d_ws) return bfail(GR_EINVAL, "null argument");
    if (bytes < B->ws_bytes) return bfail(GR_EINVAL, "workspace %zu bytes < required %zu", bytes, B->ws_bytes);
    if (reinterpret_cast<uintptr_t>(d_ws) % 256) return bfail(GR_EINVAL, "workspace not 256-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_ws) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return bfail(GR_EINVAL, "workspace is not device memory");
    }
    for (auto &ge : B->graph)
        if (ge) {
            (void)hipGraphExecDestroy(ge);
            ge = nullptr;
        }
    B->stream = reinterpret_cast<hipStream_t>(stream);
    batch_layout(B, reinterpret_cast<char *>(d_ws));
    hipStream_t s = B->stream;
    // zero the whole workspace, then upload the box table and the block tables
    const long nd = (long)(B->ws_bytes / sizeof(double));
    launch_fill(s, reinterpret_cast<double *>(d_ws), nd, 0.0);
    BLAUNCH();
    BHIP(hipMemcpyAsync(const_cast<BoxDev *>(B->D.box), B->host.data(), sizeof(BoxDev) * B->nbox,
                        hipMemcpyHostToDevice, s));
    auto up = [&](Tab &T) {
        return hipMemcpyAsync(T.dev, T.start.data(), sizeof(int) * T.start.size(), hipMemcpyHostToDevice, s);
    };
    BHIP(up(B->fine));
    BHIP(up(B->fine8));
    BHIP(up(B->norms));
    for (int d = 0; d < B->maxdepth; ++d) {
        BHIP(up(B->colour[d]));
        BHIP(up(B->cdom[d]));
        BHIP(up(B->fz[d]));
        BHIP(up(B->fz64[d]));
        BHIP(up(B->fz16[d]));
        BHIP(up(B->rr[d]));
        BHIP(up(B->colour_nf[d]));
    }
    for (auto &T : B->coefr) BHIP(up(T));
    BHIP(up(B->pfine));
    for (auto *v : {&B->pcell, &B->pfz, &B->pcellf, &B->pcoarse, &B->pcoefr, &B->pfaces, &B->colour32,
                    &B->coarse32, &B->rr32, &B->colour32nf})
        for (auto &T : *v) BHIP(up(T));
    BHIP(hipStreamSynchronize(s)); // host tables must outlive the copies
    B->D.nbox = B->nbox;
    B->Dp = B->D;
    B->Dp.partials = B->p_partials;
    B->Dp.any_active = B->p_any;
    if (B->npatch && !B->pstream) {
        BHIP(hipStreamCreateWithFlags(&B->pstream, hipStreamNonBlocking));
        BHIP(hipEventCreateWithFlags(&B->pdone, hipEventDisableTiming));
    }
    int dev = 0, khz = 0;
    BHIP(hipGetDevice(&dev));
    BHIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    B->clock_khz = khz > 0 ? khz : 100000.0;
    BHIP(hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev));
    B->qnu1 = B->qnu2 = -1; // the task table lives in the (new) workspace
    kb_queue_reset<<<1, 1024, 0, s>>>(B->qctl, B->qdone, B->nbox, 1);
    BLAUNCH();
    B->bound = true;
    return GR_OK;
}

int gr_destroy_batch(gr_batch B)
{
    if (!B) return GR_OK;
    for (auto &ge : B->graph)
        if (ge) (void)hipGraphExecDestroy(ge);
    if (B->pdone) (void)hipEventDestroy(B->pdone);
    if (B->pstream) (void)hipStreamDestroy(B->pstream);
    delete B;
    return GR_OK;
}

static double *batch_slot(gr_batch B, int item, int field)
{
    if (item < 0 || item >= B->nbox) return nullptr;
    BoxDev &X = B->host[item];
    if (field >= 0 && field < 10) return X.field[field];
    if (field >= GR_S0 && field <= GR_SM) return X.src[field - GR_S0];
    if (field == GR_AA) return X.AA;
    return nullptr;
}

int gr_batch_set_field(gr_batch B, int item, int field, const void *d_src, int dtype)
{
    if (!B || !B->bound) return bfail(B ? GR_ESTATE : GR_EINVAL, "batch not bound");
    double *dst = batch_slot(B, item, field);
    if (!dst || !d_src) return bfail(GR_EINVAL, "bad item %d / field %d / source", item, field);
    const long n = B->host[item].lev[0].n, N = n * n * n;
    if (B->host[item].patch && field < 10) { // interior of the padded iterate
        const unsigned g = (unsigned)((N + TPB - 1) / TPB);
        if (dtype == GR_F64) kp_pad_in<double><<<g, TPB, 0, B->stream>>>(dst, static_cast<const double *>(d_src), (int)n);
        else if (dtype == GR_F32) kp_pad_in<float><<<g, TPB, 0, B->stream>>>(dst, static_cast<const float *>(d_src), (int)n);
        else return bfail(GR_EINVAL, "bad dtype %d", dtype);
        BLAUNCH();
        return GR_OK;
    }
    if (dtype == GR_F64) launch_copy(B->stream, dst, static_cast<const double *>(d_src), N);
    else if (dtype == GR_F32) launch_convert_f32_to_f64(B->stream, dst, static_cast<const float *>(d_src), N);
    else return bfail(GR_EINVAL, "bad dtype %d", dtype);
    BLAUNCH();
    return GR_OK;
}

int gr_batch_get_field(gr_batch B, int item, int field, void *d_dst, int dtype)
{
    if (!B || !B->bound) return bfail(B ? GR_ESTATE : GR_EINVAL, "batch not bound");
    double *src = batch_slot(B, item, field);
    if (!src || !d_dst) return bfail(GR_EINVAL, "bad item %d / field %d / destination", item, field);
    const long n = B->host[item].lev[0].n, N = n * n * n;
    if (B->host[item].patch && field < 10) {
        const unsigned g = (unsigned)((N + TPB - 1) / TPB);
        if (dtype == GR_F64) kp_pad_out<double><<<g, TPB, 0, B->stream>>>(static_cast<double *>(d_dst), src, (int)n);
        else if (dtype == GR_F32) kp_pad_out<float><<<g, TPB, 0, B->stream>>>(static_cast<float *>(d_dst), src, (int)n);
        else return bfail(GR_EINVAL, "bad dtype %d", dtype);
        BLAUNCH();
        return GR_OK;
    }
    if (dtype == GR_F64) launch_copy(B->stream, static_cast<double *>(d_dst), src, N);
    else if (dtype == GR_F32) launch_convert_f64_to_f32(B->stream, static_cast<float *>(d_dst), src, N);
    else return bfail(GR_EINVAL, "bad dtype %d", dtype);
    BLAUNCH();
    return GR_OK;
}

int gr_batch_autotune(gr_batch B, char *report, size_t report_bytes)
{
    if (!B || !B->bound) return bfail(B ? GR_ESTATE : GR_EINVAL, "batch not bound");
    hipStream_t s = B->stream;
    const auto &H = B->host;
    // the sweeps run on field b of the boxes and their level scratch: keep b in
    // the (then unused) first shift-source array and restore it afterwards
    for (int b = 0; b < B->nper; ++b) launch_copy(s, H[b].fB[0], H[b].field[GR_BB], (long)H[b].lev[0].n * H[b].lev[0].n * H[b].lev[0].n);
    kb_begin_field<<<1, 1024, 0, s>>>(B->D, GR_BB, 0, B->nper, GR_BB); // every box active
    BLAUNCH();
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    auto upload = [&](int d) {
        hipError_t e = hipSuccess;
        for (Tab *T : {&B->fz[d], &B->fz64[d], &B->fz16[d], &B->colour_nf[d], &B->colour32nf[d]})
            if (e == hipSuccess)
                e = hipMemcpyAsync(T->dev, T->start.data(), sizeof(int) * T->start.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s); // the host tables change next
        return e;
    };
    std::string rep;
    int st = GR_OK;
    for (int d = 0; d < B->maxdepth && st == GR_OK; ++d) {
        std::vector<signed char> base = B->form[d];
        std::vector<int> sides;
        for (int b = 0; b < B->nper; ++b)
            if (base[b] >= 0) {
                const int n = H[b].lev[d].n;
                if (n >= 32 && n % 16 == 0 && std::find(sides.begin(), sides.end(), n) == sides.end()) sides.push_back(n);
            }
        std::sort(sides.begin(), sides.end());
        std::vector<signed char> best = base;
        for (int n : sides) {
            int best_form = -1;
            float best_us = 0.f;
            for (int form = 0; form <= 3 && st == GR_OK; ++form) {
                if ((form == 1 && (n < 64 || n % 32)) || (form == 2 && (n < 64 || n % 64))) continue;
                auto &F = B->form[d];
                for (int b = 0; b < B->nper; ++b) F[b] = (base[b] >= 0 && H[b].lev[d].n == n) ? form : -1;
                for (int b = B->nper; b < B->nbox; ++b) F[b] = -1;
                smooth_tabs(B, d);
                hipError_t e = upload(d);
                if (e != hipSuccess) {
                    st = bfail(GR_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
                    break;
                }
                batch_smooth(B, GR_KIND_POISSON, d, GR_BB, 2);
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < 3; ++r) batch_smooth(B, GR_KIND_POISSON, d, GR_BB, 2);
                (void)hipEventRecord(e1, s);
                e = hipEventSynchronize(e1);
                if (e != hipSuccess) {
                    st = bfail(GR_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const float us = ms * 1e3f / 3.f;
                if (best_form < 0 || us < best_us) {
                    best_form = form;
                    best_us = us;
                }
            }
            if (st != GR_OK) break;
            for (int b = 0; b < B->nper; ++b)
                if (base[b] >= 0 && H[b].lev[d].n == n) best[b] = (signed char)best_form;
            static const char *const names[4] = {"colour", "fused32x16", "fused64x16", "fused16x16"};
            char line[128];
            std::snprintf(line, sizeof line, "depth=%d n=%d form=%s us=%.2f\n", d, n, names[best_form], best_us);
            rep += line;
        }
        B->form[d] = best;
        smooth_tabs(B, d);
        if (st == GR_OK) {
            hipError_t e = upload(d);
            if (e != hipSuccess) st = bfail(GR_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int b = 0; b < B->nper; ++b) launch_copy(s, H[b].field[GR_BB], H[b].fB[0], (long)H[b].lev[0].n * H[b].lev[0].n * H[b].lev[0].n);
    BLAUNCH();
    // every captured cycle (boxes, patches, mixed-precision boxes) holds the old
    // launch shapes and tables
    for (auto &ge : B->graph)
        if (ge) {
            (void)hipGraphExecDestroy(ge);
            ge = nullptr;
        }
    B->tune_report = rep;
    if (report && report_bytes) std::snprintf(report, report_bytes, "%s", rep.c_str());
    return st;
}

int gr_batch_mixed_fallbacks(gr_batch B, int *h_flags)
{
    if (!B || !h_flags) return bfail(GR_EINVAL, "null argument");
    for (int b = 0; b < B->nbox; ++b)
        for (int f = 0; f < 10; ++f)
            h_flags[b * 10 + f] = B->fb_hist.empty() ? 0 : B->fb_hist[(size_t)b * 10 + f];
    return GR_OK;
}

int gr_batch_debug_boundary(gr_batch B, int item, int field, int level, double *d_dst)
{
    if (!B || !B->bound) return bfail(B ? GR_ESTATE : GR_EINVAL, "batch not bound");
    if (item < B->nper || item >= B->nbox || field < 0 || field >= 10 || !d_dst)
        return bfail(GR_EINVAL, "bad patch item %d / field %d / destination", item, field);
    const BoxDev &X = B->host[item];
    if (level < 0 || level >= X.nlev) return bfail(GR_EINVAL, "level %d outside 0..%d", level, X.nlev - 1);
    hipStream_t s = B->stream;
    kb_activate_depth<<<1, 1024, 0, s>>>(B->Dp, B->nper, B->nbox, -1); // the face kernel serves active patches
    patch_faces(B, s, field);
    const long w = X.lev[level].n + 2;
    launch_copy(s, d_dst, level == 0 ? X.field[field] : X.lev[level].phi, w * w * w);
    BLAUNCH();
    return GR_OK;
}

// the whole batch, or (patches_only) the patches alone from the boxes' kept fields
static int batch_solve_impl(gr_batch B, const gr_solve_opts *o, int *cycles, double *rel_res, double *item_seconds,
                            bool patches_only)
{
    b_err.clear(); // a message left by an earlier call must not be reported for this one
    if (!B || !o) return bfail(GR_EINVAL, "null argument");
    if (!B->bound) return bfail(GR_ESTATE, "batch not bound");
    if (patches_only && B->npatch == 0) return bfail(GR_EINVAL, "the batch has no patches");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 64 || o->nu2 > 64 || o->max_cycles < 0 || o->max_cycles > 100000)
        return bfail(GR_EINVAL, "bad cycle options");
    if (o->precision != GR_FP64 && o->precision != GR_MIXED) return bfail(GR_EINVAL, "bad precision");
    if (o->guess != GR_GUESS_ZERO && o->guess != GR_GUESS_CURRENT) return bfail(GR_EINVAL, "bad guess mode");
    hipStream_t s = B->stream;
    const gr_params &P = B->prm;
    const unsigned mask = o->field_mask;
    const OpConst oc = opc(B);
    const int FT = B->fine.total();
    if (!patches_only || B->rel_hist.size() != (size_t)B->nbox * 10) {
        B->rel_hist.assign((size_t)B->nbox * 10, 0.0);
        B->fb_hist.assign((size_t)B->nbox * 10, 0);
    }
    std::vector<int> zero(B->nbox, 0);
    BHIP(hipMemcpyAsync(B->D.status, zero.data(), sizeof(int) * B->nbox, hipMemcpyHostToDevice, s));
    std::vector<unsigned long long> tz((size_t)B->nbox * 10, 0ull);
    BHIP(hipMemcpyAsync(B->D.t_done, tz.data(), sizeof(unsigned long long) * tz.size(), hipMemcpyHostToDevice, s));
    const int PT = B->pfine.total();
    if (o->guess == GR_GUESS_ZERO)
        for (int f = 0; f < 10; ++f)
            if (mask & (1u << f)) {
                if (!patches_only) kb_fill_field<<<FT, TPB, 0, s>>>(B->D, B->fine.dev, f);
                if (PT) kp_fill_field<<<PT, TPB, 0, s>>>(B->Dp, B->pfine.dev, f);
            }
    BLAUNCH();
    // the patches' stream: their own, joined to the batch's by events, or the batch's
    const bool conc = !patches_only && B->npatch && B->conc && B->pstream && s != nullptr;
    hipStream_t ps = conc ? B->pstream : s;
    auto build = [&](int what, int comp) {
        kb_build<<<FT, TPB, 0, s>>>(B->D, B->fine.dev, what, comp, P.a, P.omega_m, P.c_tilde);
    };
    auto pbuild = [&](int what, int comp) {
        if (PT) kp_build<<<PT, TPB, 0, ps>>>(B->Dp, B->pfine.dev, what, comp, P.a, P.omega_m, P.c_tilde);
    };
    // the ten solves in the order of the solution scheme; the patches' builders
    // and solve of each field read their parents' solved field (and A_ij)
    struct Step {
        int kind, fid;
        std::function<void()> pre_box, pre_patch;
    };
    const std::vector<Step> steps = {
        {GR_KIND_POISSON, GR_VX, [&] {
             kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, 0, 4, oc, 0);
             kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_TMP, -1, 0, 0);
             build(0, 0);
         }, [&] { pbuild(0, 0); }},
        {GR_KIND_POISSON, GR_VY, [&] {
             kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, 0, 5, oc, 0);
             kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_TMP, -1, 0, 0);
             build(0, 1);
         }, [&] { pbuild(0, 1); }},
        {GR_KIND_POISSON, GR_VZ, [&] {
             kb_sum<kSumPPT><<<B->fine8.total(), TPB, 0, s>>>(B->D, B->fine8.dev, 0, 6, oc, 0);
             kb_finalize<<<B->nper, TPB, 0, s>>>(B->D, B->fine8.dev, 1, B_TMP, -1, 0, 0);
             build(0, 2);
         }, [&] { pbuild(0, 2); }},
        {GR_KIND_POISSON, GR_U, [&] { build(1, 0); }, [&] { pbuild(1, 0); }},
        {GR_KIND_HAMILTONIAN, GR_PSI, [&] { build(2, 0); }, [&] { pbuild(2, 0); }},
        {GR_KIND_CMC, GR_XI, [&] { build(3, 0); }, [&] { pbuild(3, 0); }},
        {GR_KIND_POISSON, GR_BX, [&] {
             build(4, 0);
             build(6, 0);
         }, [&] {
             pbuild(4, 0);
             pbuild(6, 0);
         }},
        {GR_KIND_POISSON, GR_BY, [&] { build(6, 1); }, [&] { pbuild(6, 1); }},
        {GR_KIND_POISSON, GR_BZ, [&] { build(6, 2); }, [&] { pbuild(6, 2); }},
        {GR_KIND_POISSON, GR_BB, [&] { build(5, 0); }, [&] { pbuild(5, 0); }},
    };
    auto patch_step = [&](const Step &S) -> int {
        S.pre_patch();
        BLAUNCH();
        if (mask & (1u << S.fid)) BCHK(patch_field(B, ps, S.kind, S.fid, *o));
        return GR_OK;
    };
    // concurrent patches: a host thread follows the boxes field by field.  A
    // box solve returns after synchronising the batch's stream, so once a step
    // is marked ready its fields are complete on the device and the patches'
    // stream needs no device-side wait (an event wait could also collide with
    // the box thread's graph capture of its next field)
    std::mutex mu;
    std::condition_variable cv;
    int ready = -1;      // last step whose box work is complete
    bool abort = false;  // the box thread failed
    int pstatus = GR_OK;
    std::string perr;
    std::thread worker;
    int dev = 0;
    BHIP(hipGetDevice(&dev));
    if (conc) {
        worker = std::thread([&] {
            if (hipSetDevice(dev) != hipSuccess) {
                pstatus = GR_EDEVICE;
                perr = "patch thread: hipSetDevice failed";
                return;
            }
            for (size_t k = 0; k < steps.size(); ++k) {
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return ready >= (int)k || abort; });
                    if (abort) return;
                }
                const int st = patch_step(steps[k]);
                if (st != GR_OK) {
                    pstatus = st;
                    perr = b_err;
                    return;
                }
            }
            if (hipEventRecord(B->pdone, ps) != hipSuccess) {
                pstatus = GR_EDEVICE;
                perr = "patch stream: event record failed";
            }
        });
    }
    int bstatus = GR_OK;
    for (size_t k = 0; k < steps.size() && bstatus == GR_OK && patches_only; ++k)
        bstatus = patch_step(steps[k]); // a sub-step of the refined levels: the boxes' fields are kept
    for (size_t k = 0; k < steps.size() && bstatus == GR_OK && !patches_only; ++k) {
        const Step &S = steps[k];
        S.pre_box();
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) bstatus = bfail(GR_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
        if (bstatus == GR_OK && (mask & (1u << S.fid)))
            bstatus = o->precision == GR_MIXED ? batch_field_mixed(B, S.kind, S.fid, *o) : batch_field(B, S.kind, S.fid, *o);
        if (bstatus != GR_OK) break;
        if (conc) {
            if (!(mask & (1u << S.fid))) { // no solve synchronised the stream
                e = hipStreamSynchronize(s);
                if (e != hipSuccess) {
                    bstatus = bfail(GR_EDEVICE, "stream sync: %s", hipGetErrorString(e));
                    break;
                }
            }
            std::lock_guard<std::mutex> lk(mu);
            ready = (int)k;
            cv.notify_all();
        } else if (B->npatch) {
            bstatus = patch_step(S);
        }
    }
    if (conc) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (bstatus != GR_OK) abort = true;
            cv.notify_all();
        }
        worker.join();
        if (bstatus != GR_OK || pstatus != GR_OK) {
            (void)hipStreamSynchronize(ps); // nothing of the patches may still run on return
            if (bstatus == GR_OK) {
                b_err = perr;
                return pstatus;
            }
        } else {
            BHIP(hipStreamWaitEvent(s, B->pdone, 0));
        }
    }
    if (bstatus != GR_OK) return bstatus;
    BLAUNCH();
    // results
    std::vector<int> st(B->nbox), cyc((size_t)B->nbox * 10);
    std::vector<unsigned long long> td((size_t)B->nbox * 10), t0(20);
    BHIP(hipMemcpyAsync(st.data(), B->D.status, sizeof(int) * st.size(), hipMemcpyDeviceToHost, s));
    BHIP(hipMemcpyAsync(cyc.data(), B->D.cycles, sizeof(int) * cyc.size(), hipMemcpyDeviceToHost, s));
    BHIP(hipMemcpyAsync(td.data(), B->D.t_done, sizeof(unsigned long long) * td.size(), hipMemcpyDeviceToHost, s));
    BHIP(hipMemcpyAsync(t0.data(), B->D.t_start, sizeof(unsigned long long) * 20, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (cycles) std::memcpy(cycles, cyc.data(), sizeof(int) * cyc.size());
    if (item_seconds)
        for (int b = 0; b < B->nbox; ++b) {
            double sum = 0.0;
            const int ts = B->host[b].patch ? 10 : 0;
            for (int f = 0; f < 10; ++f)
                if ((mask & (1u << f)) && td[b * 10 + f] >= t0[ts + f]) sum += (double)(td[b * 10 + f] - t0[ts + f]);
            item_seconds[b] = sum / (B->clock_khz * 1e3);
        }
    if (rel_res) {
        for (int b = 0; b < B->nbox; ++b)
            for (int f = 0; f < 10; ++f) rel_res[b * 10 + f] = B->rel_hist[(size_t)b * 10 + f];
    }
    int first_bad = GR_OK;
    for (int b = 0; b < B->nbox; ++b)
        if (st[b] != GR_OK) {
            first_bad = st[b];
            bfail(st[b], "item %d did not converge (status %d)", b, st[b]);
            break;
        }
    return first_bad;
}

int gr_batch_solve(gr_batch B, const gr_solve_opts *o, int *cycles, double *rel_res, double *item_seconds)
{
    return batch_solve_impl(B, o, cycles, rel_res, item_seconds, false);
}

int gr_batch_solve_patches(gr_batch B, const gr_solve_opts *o, int *cycles, double *rel_res, double *item_seconds)
{
    return batch_solve_impl(B, o, cycles, rel_res, item_seconds, true);
}

} // extern "C"
