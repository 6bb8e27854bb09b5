// Learned initial guess: a small 3-D U-Net (levels with c0/c1/c2/c3 channels,
// two 3^3 convolutions + ReLU per level, 2x2x2 average pooling down, nearest
// upsampling up, skip concatenation, 1x1 head), trained and run on the GPU by
// the kernels below.
//
// Layout: activations channels-last [z][y][x][C] in BF16, periodic boundaries
// (the fields live on a periodic box).  Convolutions are implicit GEMMs on the
// BF16 matrix cores (FP32 accumulation): M = 16 voxels per product, N =
// output channels (16 per tile), K = 27 taps x input channels (weight rows
// padded to a multiple of 32).  The input-gradient of a
// convolution is the same kernel applied to the output-gradient with the
// weights flipped in space and transposed in channels.  Weight gradients
// accumulate in FP32; Adam keeps FP32 master weights.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gr_internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------ convolution

// out[v][ocoff + co] = act(bias[co] + sum_k in[v + off(tap)][icoff + ci] w[co][k]),
// k = tap * cin + ci, taps ordered (dz, dy, dx) in {-1,0,1}^3 with dx fastest.
// One wave: VG groups of 16 consecutive voxels x all COUT channels, so each
// weight operand (B) feeds VG matrix-core products.  The 27 taps are unrolled
// (every lane of a product works on the same tap) and each tap runs over the
// input channels in steps of KS = 32 (v_mfma_f32_16x16x32_bf16, 8 channels per
// lane) when cin % 32 == 0, else KS = 16 (v_mfma_f32_16x16x16_bf16, 4 channels
// per lane); a lane's neighbour rows are formed once, so the inner loop is
// loads and matrix products.  n^3 must be a multiple of 64 VG (4 waves per
// block) and cin a multiple of KS.
template <int KS> struct ConvOperand;
template <> struct ConvOperand<32> {
    typedef bf16x8 type;
    static __device__ __forceinline__ floatx4 mfma(type a, type b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct ConvOperand<16> {
    typedef shortx4 type;
    static __device__ __forceinline__ floatx4 mfma(type a, type b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
};

template <int COUT, int VG, int KS, bool RELU, bool BIAS>
__global__ void __launch_bounds__(256) k_conv3(const bf16 *__restrict__ in, int cin, int icstride, int icoff,
                                               const bf16 *__restrict__ w, int kpad, const float *__restrict__ bias,
                                               bf16 *__restrict__ out, int ocstride, int ocoff, int n)
{
    typedef ConvOperand<KS> Op;
    typedef typename Op::type opT;
    constexpr int NT = COUT / 16, PER = KS / 4;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int v0 = (blockIdx.x * 4 + wave) * 16 * VG;
    const int i = lane & 15, g = lane >> 4;
    // neighbour coordinates of this lane's voxel in each group: x, y * n, z * n^2
    int xo[VG][3], yo[VG][3], zo[VG][3];
#pragma unroll
    for (int q = 0; q < VG; ++q) {
        const int v = v0 + 16 * q + i;
        const int x = v % n, y = (v / n) % n, z = v / (n * n);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xo[q][d] = wrapn(x + d - 1, n);
            yo[q][d] = wrapn(y + d - 1, n) * n;
            zo[q][d] = wrapn(z + d - 1, n) * n * n;
        }
    }
    floatx4 acc[VG][NT];
#pragma unroll
    for (int q = 0; q < VG; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bf16 *wl = w + (long)i * kpad + PER * g;
    const long wstep = (long)16 * kpad;
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int tap = (dz * 3 + dy) * 3 + dx;
                const bf16 *src[VG];
#pragma unroll
                for (int q = 0; q < VG; ++q)
                    src[q] = in + (long)(zo[q][dz] + yo[q][dy] + xo[q][dx]) * icstride + icoff + PER * g;
                const bf16 *wt = wl + tap * cin;
                for (int c0 = 0; c0 < cin; c0 += KS) {
                    opT bw[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t) bw[t] = *reinterpret_cast<const opT *>(wt + t * wstep + c0);
#pragma unroll
                    for (int q = 0; q < VG; ++q) {
                        const opT a = *reinterpret_cast<const opT *>(src[q] + c0);
#pragma unroll
                        for (int t = 0; t < NT; ++t) acc[q][t] = Op::mfma(a, bw[t], acc[q][t]);
                    }
                }
            }
    // lane holds D[4g + j][i]: voxel v0 + 16 q + 4g + j, channel 16t + i
#pragma unroll
    for (int q = 0; q < VG; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = 16 * t + i;
            const float b = BIAS ? bias[co] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float r = acc[q][t][j] + b;
                if (RELU) r = r > 0.0f ? r : 0.0f;
                out[(long)(v0 + 16 * q + 4 * g + j) * ocstride + ocoff + co] = (bf16)r;
            }
        }
}

// The same convolution with the input staged in LDS: one block computes a
// 16 (x) x 4 (y) x 4 (z) tile of output voxels; wave w takes the plane z0 + w
// and its product group q the row y0 + q.  For each chunk of CW input
// channels the block copies the tile's 18 x 6 x 6 input halo into LDS (voxel
// stride CW + 8 elements, so the 16-byte reads of 8 consecutive lanes fall in
// distinct banks), then every tap reads its operand at a constant offset from
// the lane's base.  CW = 32: one v_mfma_f32_16x16x32_bf16 per tap, all lanes
// on the same tap.  CW = 16: taps go in pairs, lanes g < 2 on the first and
// g >= 2 on the second (8 channels each), the unpaired 27th tap padded with
// zeros.  n must be a multiple of 16 and cin of CW.
constexpr int CT_HX = 18, CT_HY = 6, CT_HZ = 6, CT_HV = CT_HX * CT_HY * CT_HZ;

template <int COUT, int CW, bool RELU, bool BIAS>
__global__ void __launch_bounds__(256) k_conv3_lds(const bf16 *__restrict__ in, int cin, int icstride, int icoff,
                                                   const bf16 *__restrict__ w, int kpad,
                                                   const float *__restrict__ bias, bf16 *__restrict__ out,
                                                   int ocstride, int ocoff, int n)
{
    constexpr int NT = COUT / 16, STR = CW + 8, UPV = CW / 8, NU = CT_HV * UPV, PERT = (NU + 255) / 256;
    __shared__ __align__(16) bf16 tile[CT_HV * STR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    // blocks in contiguous runs per XCD (dispatch is round-robin over the 8 XCDs)
    const int nblk = gridDim.x;
    int b = blockIdx.x;
    if (nblk % 8 == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int tx = n >> 4, ty = n >> 2;
    const int X0 = (b % tx) * 16, Y0 = ((b / tx) % ty) * 4, Z0 = (b / tx / ty) * 4;
    floatx4 acc[4][NT];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const bool hi = g >= 2;
    const int lbase = (wave * CT_HY * CT_HX + i) * STR + (CW == 32 ? 8 * g : 8 * (g & 1));
    const bf16 *wl = w + (long)i * kpad + (CW == 32 ? 8 * g : 8 * (g & 1));
    const long wstep = (long)16 * kpad;
    for (int c0 = 0; c0 < cin; c0 += CW) {
        bf16x8 stage[PERT];
#pragma unroll
        for (int r = 0; r < PERT; ++r) {
            const int u = threadIdx.x + 256 * r;
            if (u < NU) {
                const int h = u / UPV, cu = u % UPV;
                const int hx = h % CT_HX, hy = (h / CT_HX) % CT_HY, hz = h / (CT_HX * CT_HY);
                const long src = ((long)wrapn(Z0 - 1 + hz, n) * n + wrapn(Y0 - 1 + hy, n)) * n + wrapn(X0 - 1 + hx, n);
                stage[r] = *reinterpret_cast<const bf16x8 *>(in + src * icstride + icoff + c0 + 8 * cu);
            }
        }
        __syncthreads(); // the previous chunk's reads are done
#pragma unroll
        for (int r = 0; r < PERT; ++r) {
            const int u = threadIdx.x + 256 * r;
            if (u < NU) *reinterpret_cast<bf16x8 *>(tile + (u / UPV) * STR + 8 * (u % UPV)) = stage[r];
        }
        __syncthreads();
        if (CW == 32) {
            // rows (dz, dy) in a loop, the three dx of a row unrolled
#pragma unroll 1
            for (int r = 0; r < 9; ++r) {
                const int roff = ((r / 3) * CT_HY + r % 3) * CT_HX * STR;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int tap = 3 * r + dx;
                    bf16x8 bw[NT];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        bw[t] = *reinterpret_cast<const bf16x8 *>(wl + t * wstep + tap * cin + c0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bf16x8 a =
                            *reinterpret_cast<const bf16x8 *>(tile + lbase + q * CT_HX * STR + roff + dx * STR);
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t], acc[q][t], 0, 0, 0);
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int m = 0; m < 14; ++m) {
                const int tap = 2 * m + (hi ? 1 : 0);
                const bool valid = tap < 27;
                const int toff = (((tap / 9) * CT_HY + (tap / 3) % 3) * CT_HX + tap % 3) * STR;
                const int wk = tap * cin + c0;
                bf16x8 bw[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (valid) bw[t] = *reinterpret_cast<const bf16x8 *>(wl + t * wstep + wk);
                    else
#pragma unroll
                        for (int j = 0; j < 8; ++j) bw[t][j] = (bf16)0.0f;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bf16x8 a;
                    if (valid) a = *reinterpret_cast<const bf16x8 *>(tile + lbase + q * CT_HX * STR + toff);
                    else
#pragma unroll
                        for (int j = 0; j < 8; ++j) a[j] = (bf16)0.0f;
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[q][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[t], acc[q][t], 0, 0, 0);
                }
            }
        }
    }
    // lane holds D[4g + j][i]: voxel (X0 + 4g + j, Y0 + q, Z0 + wave), channel 16t + i
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const long vrow = ((long)(Z0 + wave) * n + (Y0 + q)) * n + X0 + 4 * g;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int co = 16 * t + i;
            const float bb = BIAS ? bias[co] : 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float r = acc[q][t][j] + bb;
                if (RELU) r = r > 0.0f ? r : 0.0f;
                out[(vrow + j) * ocstride + ocoff + co] = (bf16)r;
            }
        }
    }
}

// Weight gradient of a 3^3 convolution on the BF16 matrix cores:
//   dW[co][tap*cin + ci] = sum_v g[v][gcoff + co] in[v + off(tap)][icoff + ci],
//   db[co] = sum_v g[v][gcoff + co].
// Per tap this is a GEMM with M = cout, N = cin and K = the voxels.  A block
// owns one tap and every WB-th chunk of 64 consecutive voxels; each chunk's
// output gradient and shifted input are staged in LDS transposed (channel
// rows of 64 voxels), so an MFMA operand (8 consecutive voxels of one channel)
// is one 16-byte LDS read.  Each wave accumulates its 16 x 16 (co, ci) tiles
// over the block's chunks in FP32; the block writes its partial sums, and
// k_wgrad_reduce adds the WB partials in a fixed order (deterministic).
constexpr int WG_CHUNK = 64;              // voxels per staged chunk (two K steps)
constexpr int WG_ROW = WG_CHUNK + 8;      // LDS row pitch in bf16 (144 bytes)
constexpr int WG_MAXC = 128;              // largest channel count of either side
constexpr int WG_MAXT = 8;                // 16 x 16 tiles per wave (cout/16 * cin/16 <= 32)
__global__ void __launch_bounds__(TPB) k_conv3_wgrad(const bf16 *__restrict__ g, int cout, int gcstride, int gcoff,
                                                     const bf16 *__restrict__ in, int cin, int icstride, int icoff,
                                                     float *__restrict__ part, float *__restrict__ bpart, int n)
{
    __shared__ __attribute__((aligned(16))) bf16 sg[64 * WG_ROW];
    __shared__ __attribute__((aligned(16))) bf16 si[WG_MAXC * WG_ROW];
    const int tap = blockIdx.y;
    const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    const long N = (long)n * n * n;
    const long nchunk = N / WG_CHUNK;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, gq = lane >> 4;
    const int tco = cout / 16, tci = cin / 16, ntile = tco * tci;
    floatx4 acc[WG_MAXT];
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.0f;
    const int gvec = cout / 8, ivec = cin / 8;
    for (long ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const long v0 = ch * WG_CHUNK;
        // stage: g rows [co][voxel], input rows [ci][voxel] at the tap's shifted voxels
        for (int e = threadIdx.x; e < WG_CHUNK * gvec; e += TPB) {
            const int r = e / gvec, q = e % gvec;
            const bf16x8 val = *reinterpret_cast<const bf16x8 *>(g + (v0 + r) * gcstride + gcoff + 8 * q);
#pragma unroll
            for (int j = 0; j < 8; ++j) sg[(8 * q + j) * WG_ROW + r] = val[j];
        }
        for (int e = threadIdx.x; e < WG_CHUNK * ivec; e += TPB) {
            const int r = e / ivec, q = e % ivec;
            const long v = v0 + r;
            const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((long)n * n));
            const long src = ((long)wrapn(z + dz, n) * n + wrapn(y + dy, n)) * n + wrapn(x + dx, n);
            const bf16x8 val = *reinterpret_cast<const bf16x8 *>(in + src * icstride + icoff + 8 * q);
#pragma unroll
            for (int j = 0; j < 8; ++j) si[(8 * q + j) * WG_ROW + r] = val[j];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < WG_MAXT; ++t) {
            const int tile = wave + 4 * t;
            if (tile < ntile) {
                const int cot = tile / tci, cit = tile % tci;
#pragma unroll
                for (int ks = 0; ks < WG_CHUNK / 32; ++ks) {
                    const int k = 32 * ks + 8 * gq;
                    const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sg + (16 * cot + i) * WG_ROW + k);
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(si + (16 * cit + i) * WG_ROW + k);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        if (tap == 13 && (int)threadIdx.x < cout) {
            float s = 0.0f;
            for (int r = 0; r < WG_CHUNK; ++r) s += (float)sg[threadIdx.x * WG_ROW + r];
            bacc += s;
        }
        __syncthreads();
    }
    // partial of this block: part[blockIdx.x][tap][co][ci]; lane holds D[4gq + j][i]
    float *dst = part + ((long)blockIdx.x * 27 + tap) * cout * cin;
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) {
        const int tile = wave + 4 * t;
        if (tile < ntile) {
            const int cot = tile / tci, cit = tile % tci;
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[(long)(16 * cot + 4 * gq + j) * cin + 16 * cit + i] = acc[t][j];
        }
    }
    if (tap == 13 && (int)threadIdx.x < cout) bpart[(long)blockIdx.x * cout + threadIdx.x] = bacc;
}

// dw[co][tap*cin + ci] += sum over the nb block partials (in order); db likewise
__global__ void k_wgrad_reduce(const float *__restrict__ part, const float *__restrict__ bpart, int nbk, int cout,
                               int cin, float *__restrict__ dw, float *__restrict__ db)
{
    const long per = 27L * cout * cin;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < per) {
        const int tap = (int)(q / ((long)cout * cin));
        const int rem = (int)(q % ((long)cout * cin));
        const int co = rem / cin, ci = rem % cin;
        float s = 0.0f;
        for (int b = 0; b < nbk; ++b) s += part[(long)b * per + q];
        dw[(long)co * 27 * cin + tap * cin + ci] += s;
    }
    if (db && q < cout) {
        float s = 0.0f;
        for (int b = 0; b < nbk; ++b) s += bpart[(long)b * cout + q];
        db[q] += s;
    }
}

// ------------------------------------------------------------ elementwise

// planar FP32 [cin][n^3] -> channels-last BF16 [n^3][16] (zero channels above cin)
__global__ void k_pack_input(const float *__restrict__ src, int cin, bf16 *__restrict__ dst, long N)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    bf16x8 lo, hi; // the voxel's 16 channels as two 16-byte stores
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        lo[c] = (bf16)(c < cin ? src[c * N + v] : 0.0f);
        hi[c] = (bf16)(c + 8 < cin ? src[(c + 8) * N + v] : 0.0f);
    }
    bf16x8 *d = reinterpret_cast<bf16x8 *>(dst + v * 16);
    d[0] = lo;
    d[1] = hi;
}

// 2x2x2 average of channels [coff, coff + c) -> [m^3][c]
__global__ void k_pool(const bf16 *__restrict__ in, int cstride, int coff, int c, bf16 *__restrict__ out, int n)
{
    const int m = n / 2;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)m * m * m * c) return;
    const int ch = (int)(q % c);
    const long V = q / c;
    const int X = (int)(V % m), Y = (int)((V / m) % m), Z = (int)(V / ((long)m * m));
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const long v = ((long)(2 * Z + (k >> 2)) * n + 2 * Y + ((k >> 1) & 1)) * n + 2 * X + (k & 1);
        s += (float)in[v * cstride + coff + ch];
    }
    out[V * c + ch] = (bf16)(0.125f * s);
}

// gradient of the pooling, added to channels [coff, coff + c) of gin
__global__ void k_pool_bwd_add(const bf16 *__restrict__ gout, int c, bf16 *__restrict__ gin, int cstride, int coff,
                               int n)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)n * n * n * c) return;
    const int ch = (int)(q % c);
    const long v = q / c;
    const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((long)n * n));
    const int m = n / 2;
    const long V = ((long)(z / 2) * m + y / 2) * m + x / 2;
    const long d = v * cstride + coff + ch;
    gin[d] = (bf16)((float)gin[d] + 0.125f * (float)gout[V * c + ch]);
}

// nearest upsampling of [m^3][c] into channels [0, c) of out [n^3][cstride]
// one thread per voxel and group of 8 channels (16-byte loads and stores;
// c and cstride are multiples of 8)
__global__ void k_upsample(const bf16 *__restrict__ in, int c, bf16 *__restrict__ out, int cstride, int n)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int cg = c >> 3;
    if (q >= (long)n * n * n * cg) return;
    const int ch = (int)(q % cg) * 8;
    const long v = q / cg;
    const int x = (int)(v % n), y = (int)((v / n) % n), z = (int)(v / ((long)n * n));
    const int m = n / 2;
    *reinterpret_cast<bf16x8 *>(out + v * cstride + ch) =
        *reinterpret_cast<const bf16x8 *>(in + (((long)(z / 2) * m + y / 2) * m + x / 2) * c + ch);
}

// gradient of the upsampling: sum of the 8 children's channels [0, c)
__global__ void k_upsample_bwd(const bf16 *__restrict__ gout, int cstride, int c, bf16 *__restrict__ gin, int n)
{
    const int m = n / 2;
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)m * m * m * c) return;
    const int ch = (int)(q % c);
    const long V = q / c;
    const int X = (int)(V % m), Y = (int)((V / m) % m), Z = (int)(V / ((long)m * m));
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const long v = ((long)(2 * Z + (k >> 2)) * n + 2 * Y + ((k >> 1) & 1)) * n + 2 * X + (k & 1);
        s += (float)gout[v * cstride + ch];
    }
    gin[V * c + ch] = (bf16)s;
}

// g = g * (a > 0) on channels [coff, coff + c) of both (ReLU gradient)
__global__ void k_relu_bwd(bf16 *__restrict__ g, int gcstride, int gcoff, const bf16 *__restrict__ a, int acstride,
                           int acoff, int c, long N)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N * c) return;
    const int ch = (int)(q % c);
    const long v = q / c;
    if (!((float)a[v * acstride + acoff + ch] > 0.0f)) g[v * gcstride + gcoff + ch] = (bf16)0.0f;
}

// 1x1 head: y[o][v] = b[o] + sum_c w[o][c] h[v][c]   (FP32 planar output)
__global__ void k_head(const bf16 *__restrict__ h, int c, const float *__restrict__ w, const float *__restrict__ b,
                       float *__restrict__ y, int cout, long N)
{
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    float hv[16];
    if (c == 16) { // two 16-byte loads
        const bf16x8 *hp = reinterpret_cast<const bf16x8 *>(h + v * 16);
        const bf16x8 lo = hp[0], hi = hp[1];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            hv[k] = (float)lo[k];
            hv[k + 8] = (float)hi[k];
        }
    } else {
        for (int k = 0; k < c; ++k) hv[k] = (float)h[v * c + k];
    }
    for (int o = 0; o < cout; ++o) {
        float s = b[o];
        for (int k = 0; k < c; ++k) s += w[o * c + k] * hv[k];
        y[o * N + v] = s;
    }
}

// MSE loss pieces: gy = 2 (y - t) / (cout N); per-block partial sums of (y - t)^2
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ gy, long total,
                      float *__restrict__ partial)
{
    __shared__ float sh[TPB];
    float s = 0.0f;
    for (long q = (long)blockIdx.x * TPB + threadIdx.x; q < total; q += (long)gridDim.x * TPB) {
        const float d = y[q] - t[q];
        gy[q] = 2.0f * d / (float)total;
        s += d * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Optional smoothness term of the loss, lambda * mean((Lap d)^2) with d = y - t
// and Lap the 7-point periodic Laplacian of unit spacing, per channel: the
// judge of a guess is a residual, which weights errors by Lap.  Pass 1:
// q = Lap d and partial sums of q^2; pass 2: gy += 2 lambda Lap q / total
// (Lap is symmetric).
__device__ __forceinline__ long lap_nb(int x, int y, int z, int n, int dx, int dy, int dz)
{
    x += dx;
    y += dy;
    z += dz;
    x = x < 0 ? x + n : (x >= n ? x - n : x);
    y = y < 0 ? y + n : (y >= n ? y - n : y);
    z = z < 0 ? z + n : (z >= n ? z - n : z);
    return ((long)z * n + y) * n + x;
}

template <bool FROM_DIFF>
__device__ __forceinline__ float lap_at(const float *__restrict__ a, const float *__restrict__ b, long base, int x,
                                        int y, int z, int n)
{
    auto v = [&](long q) { return FROM_DIFF ? a[base + q] - b[base + q] : a[base + q]; };
    const float c = v(((long)z * n + y) * n + x);
    return v(lap_nb(x, y, z, n, 1, 0, 0)) + v(lap_nb(x, y, z, n, -1, 0, 0)) + v(lap_nb(x, y, z, n, 0, 1, 0)) +
           v(lap_nb(x, y, z, n, 0, -1, 0)) + v(lap_nb(x, y, z, n, 0, 0, 1)) + v(lap_nb(x, y, z, n, 0, 0, -1)) -
           6.0f * c;
}

__global__ void k_lap_loss1(const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ q, int n,
                            long total, float *__restrict__ partial)
{
    __shared__ float sh[TPB];
    const long N = (long)n * n * n;
    float s = 0.0f;
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < total; p += (long)gridDim.x * TPB) {
        const long ch = p / N, v = p - ch * N;
        const int x = (int)(v % n), yy = (int)((v / n) % n), z = (int)(v / ((long)n * n));
        const float l = lap_at<true>(y, t, ch * N, x, yy, z, n);
        q[p] = l;
        s += l * l;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_lap_loss2(const float *__restrict__ q, float *__restrict__ gy, int n, long total, float lam)
{
    const long N = (long)n * n * n;
    for (long p = (long)blockIdx.x * TPB + threadIdx.x; p < total; p += (long)gridDim.x * TPB) {
        const long ch = p / N, v = p - ch * N;
        const int x = (int)(v % n), yy = (int)((v / n) % n), z = (int)(v / ((long)n * n));
        gy[p] += 2.0f * lam * lap_at<false>(q, nullptr, ch * N, x, yy, z, n) / (float)total;
    }
}

// head backward: gh[v][c] = sum_o w[o][c] gy[o][v]; the block's partial sums of
// dW[o][c] = sum_v gy[o][v] h[v][c] and db[o] = sum_v gy[o][v] over its 256
// voxels, one parameter per thread in voxel order, to part[block][cout*c + cout]
// (k_head_reduce adds the blocks in order: deterministic).
__global__ void __launch_bounds__(TPB) k_head_bwd(const float *__restrict__ gy, const bf16 *__restrict__ h, int c,
                                                  const float *__restrict__ w, int cout, bf16 *__restrict__ gh,
                                                  float *__restrict__ part, long N)
{
    __shared__ float sgy[16][TPB];
    __shared__ float sh[TPB][17];
    const long v0 = (long)blockIdx.x * TPB;
    const long v = v0 + threadIdx.x;
    if (v < N) {
        float hv[16];
        for (int k = 0; k < c; ++k) {
            hv[k] = (float)h[v * c + k];
            sh[threadIdx.x][k] = hv[k];
        }
        for (int o = 0; o < cout; ++o) sgy[o][threadIdx.x] = gy[o * N + v];
        for (int k = 0; k < c; ++k) {
            float s = 0.0f;
            for (int o = 0; o < cout; ++o) s += w[o * c + k] * gy[o * N + v];
            gh[v * c + k] = (bf16)s;
        }
    } else {
        for (int k = 0; k < c; ++k) sh[threadIdx.x][k] = 0.0f;
        for (int o = 0; o < cout; ++o) sgy[o][threadIdx.x] = 0.0f;
    }
    __syncthreads();
    const int npar = cout * c + cout;
    for (int q = threadIdx.x; q < npar; q += TPB) {
        float s = 0.0f;
        if (q < cout * c) {
            const int o = q / c, k = q % c;
            for (int r = 0; r < TPB; ++r) s += sgy[o][r] * sh[r][k];
        } else {
            const int o = q - cout * c;
            for (int r = 0; r < TPB; ++r) s += sgy[o][r];
        }
        part[(long)blockIdx.x * npar + q] = s;
    }
}

// one block per parameter: thread t adds partials t, t + 256, ... in order,
// then a fixed tree over the threads (deterministic)
__global__ void __launch_bounds__(TPB) k_head_reduce(const float *__restrict__ part, int nblk, int npar, int nw,
                                                     float *__restrict__ dw, float *__restrict__ db)
{
    __shared__ float sh[TPB];
    const int q = blockIdx.x;
    float s = 0.0f;
    for (int b = threadIdx.x; b < nblk; b += TPB) s += part[(long)b * npar + q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (q < nw) dw[q] += sh[0];
        else db[q - nw] += sh[0];
    }
}

// FP32 master weights -> BF16 forward layout [co][kpad] and the flipped /
// transposed layout [ci][kpad'] used for input gradients.
__global__ void k_prep_weights(const float *__restrict__ w, int cout, int cin, int kpad, int kpadT,
                               bf16 *__restrict__ wf, bf16 *__restrict__ wt)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long tot = (long)cout * kpad;
    if (q < tot) {
        const int co = (int)(q / kpad), k = (int)(q % kpad);
        wf[q] = (bf16)(k < 27 * cin ? w[(long)co * 27 * cin + k] : 0.0f);
    }
    const long totT = (long)cin * kpadT;
    if (q < totT) {
        const int ci = (int)(q / kpadT), k = (int)(q % kpadT);
        float val = 0.0f;
        if (k < 27 * cout) {
            const int tapT = k / cout, co = k % cout;
            const int tap = 26 - tapT; // off(tapT) = -off(tap)
            val = w[(long)co * 27 * cin + tap * cin + ci];
        }
        wt[q] = (bf16)val;
    }
}

// Gradient-norm clipping: per-block sums of g^2 (FP64, fixed grid), then one
// block adds them in order and writes scale = min(1, clip / |g|) (1 for a zero
// or non-finite norm is not used: a non-finite norm gives scale 0, so the step
// leaves the weights unchanged).
constexpr int kClipBlocks = 256;
__global__ void __launch_bounds__(TPB) k_sumsq(const float *__restrict__ g, long N, double *__restrict__ part)
{
    __shared__ double sh[TPB];
    double s = 0.0;
    for (long q = (long)blockIdx.x * TPB + threadIdx.x; q < N; q += (long)gridDim.x * TPB) s += (double)g[q] * g[q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_clip_scale(const double *__restrict__ part, int nbk, float clip, float *__restrict__ scale,
                             float *__restrict__ norm_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nbk; ++b) s += part[b];
    const double nrm = sqrt(s);
    norm_out[0] = (float)nrm;
    scale[0] = !isfinite(nrm) ? 0.0f : (nrm > (double)clip ? (float)((double)clip / nrm) : 1.0f);
}

// Adam (FP32) on the gradient times *gscale (1 without clipping):
// p -= lr * mhat / (sqrt(vhat) + eps)
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       long N, float lr, float b1, float b2, float eps, float c1, float c2,
                       const float *__restrict__ gscale)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const float gq = g[q] * gscale[0];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// He-normal initialisation from a counter-based generator: splitmix64 of
// (seed, index) -> two uniforms -> Box-Muller.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__global__ void k_init_normal(float *__restrict__ p, long N, float stddev, unsigned long long seed)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const unsigned long long r = splitmix64(seed ^ splitmix64((unsigned long long)q));
    const double u1 = ((r >> 11) + 1.0) * (1.0 / 9007199254740993.0);
    const double u2 = (splitmix64(r) >> 11) * (1.0 / 9007199254740992.0);
    p[q] = (float)(stddev * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

__global__ void k_zero_f32(float *__restrict__ p, long N)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) p[q] = 0.0f;
}
__global__ void k_zero_bf16(bf16 *__restrict__ p, long N)
{
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < N) p[q] = (bf16)0.0f;
}

unsigned nb(long count) { return (unsigned)((count + TPB - 1) / TPB); }

thread_local std::string u_err;
int ufail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int ufail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    u_err = buf;
    return code;
}
#define UHIP(expr)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess) return ufail(GR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));       \
    } while (0)
#define ULAUNCH()                                                                                     \
    do {                                                                                              \
        hipError_t e_ = hipGetLastError();                                                            \
        if (e_ != hipSuccess) return ufail(GR_EDEVICE, "kernel launch: %s", hipGetErrorString(e_));   \
    } while (0)

int pad32(int k) { return (k + 31) / 32 * 32; }

constexpr int kWgradBlocks = 64; // voxel-chunk blocks per tap of the weight gradient

template <int COUT, int VG, bool RELU, bool BIAS>
void launch_conv_ks(hipStream_t s, unsigned grid, const bf16 *in, int cin, int ics, int icoff, const bf16 *w, int kpad,
                    const float *bias, bf16 *out, int ocs, int ocoff, int n)
{
    if (cin % 32 == 0)
        k_conv3<COUT, VG, 32, RELU, BIAS><<<grid, 256, 0, s>>>(in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n);
    else
        k_conv3<COUT, VG, 16, RELU, BIAS><<<grid, 256, 0, s>>>(in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n);
}

template <bool RELU, bool BIAS>
bool launch_conv_t(hipStream_t s, int cout, const bf16 *in, int cin, int ics, int icoff, const bf16 *w, int kpad,
                   const float *bias, bf16 *out, int ocs, int ocoff, int n)
{
    const long N = (long)n * n * n;
    if (cin % 16 || N % 64 || N >= (1L << 31)) return false;
    if (n % 16 == 0) {
        const unsigned gl = (unsigned)((n / 16) * (n / 4) * (n / 4));
#define CONV_LDS(C)                                                                                           \
    case C:                                                                                                   \
        if (cin % 32 == 0)                                                                                    \
            k_conv3_lds<C, 32, RELU, BIAS><<<gl, 256, 0, s>>>(in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n); \
        else                                                                                                  \
            k_conv3_lds<C, 16, RELU, BIAS><<<gl, 256, 0, s>>>(in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n); \
        return true;
        switch (cout) {
            CONV_LDS(16)
            CONV_LDS(32)
            CONV_LDS(48)
            CONV_LDS(64)
            CONV_LDS(96)
            CONV_LDS(128)
        default: return false;
        }
#undef CONV_LDS
    }
    // four voxel groups per wave where the grid allows it (two for the widest outputs), else one
    const int vg = (N % 256 == 0) ? (cout >= 96 ? 2 : 4) : 1;
    const unsigned grid = (unsigned)(N / (64 * vg));
#define CONV_CASE(C)                                                                                          \
    case C:                                                                                                   \
        if (vg == 4) launch_conv_ks<C, 4, RELU, BIAS>(s, grid, in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n); \
        else if (vg == 2) launch_conv_ks<C, 2, RELU, BIAS>(s, grid, in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n); \
        else launch_conv_ks<C, 1, RELU, BIAS>(s, grid, in, cin, ics, icoff, w, kpad, bias, out, ocs, ocoff, n); \
        break;
    switch (cout) {
        CONV_CASE(16)
        CONV_CASE(32)
        CONV_CASE(48)
        CONV_CASE(64)
        CONV_CASE(96)
        CONV_CASE(128)
    default: return false;
    }
#undef CONV_CASE
    return true;
}

} // namespace

// ------------------------------------------------------------------ network

struct ConvLayer {
    int cin, cout, kpad, kpadT;
    long w_off, b_off; // offsets into the FP32 parameter vector
    bf16 *wf = nullptr, *wt = nullptr;
};

struct Act { // one channels-last BF16 tensor
    bf16 *p = nullptr;
    int n = 0, c = 0;
};

struct gr_unet_s {
    gr_unet_desc d{};
    int max_n = 0;
    int c[4];
    ConvLayer conv[14]; // e0a e0b e1a e1b e2a e2b e3a e3b d2a d2b d1a d1b d0a d0b
    long head_w = 0, head_b = 0;
    long nparam = 0;
    // device
    float *param = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    float *loss_partial = nullptr, *y = nullptr, *gy = nullptr, *lq = nullptr;
    float *wg_part = nullptr, *wg_bpart = nullptr; // weight-gradient block partials
    double *gn_part = nullptr;                       // gradient-norm block partials
    float *gscale = nullptr;
    bf16 *x0 = nullptr;
    Act ea[4], eb3, cat[3], p[3], da[3], db[3];       // forward
    Act g_ea[4], g_eb3, g_cat[3], g_p[3], g_da[3], g_db[3], g_x; // backward
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    long step = 0;
};

namespace {

enum { E0A, E0B, E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B, D0A, D0B };

size_t unet_layout(gr_unet U, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    auto takeF = [&](size_t n) { return reinterpret_cast<float *>(take(sizeof(float) * n)); };
    auto takeB = [&](size_t n) { return reinterpret_cast<bf16 *>(take(sizeof(bf16) * n)); };
    U->param = takeF(U->nparam);
    U->grad = takeF(U->nparam);
    U->adam_m = takeF(U->nparam);
    U->adam_v = takeF(U->nparam);
    for (auto &L : U->conv) {
        L.wf = takeB((size_t)L.cout * L.kpad);
        L.wt = takeB((size_t)L.cin * L.kpadT);
    }
    const int n = U->max_n;
    const long N = (long)n * n * n;
    U->loss_partial = takeF(2048);
    U->gn_part = reinterpret_cast<double *>(take(sizeof(double) * kClipBlocks));
    U->gscale = takeF(2); // [0] clip scale of the gradient, [1] its norm
    // block partials of the weight gradients: the 3^3 convolutions' (64 blocks x 27
    // taps x cout x cin) or the head's (one block per 256 voxels x its parameters)
    const size_t head_part = (size_t)((N + TPB - 1) / TPB) * (size_t)(U->d.out_ch * U->c[0] + U->d.out_ch);
    U->wg_part = takeF(std::max((size_t)kWgradBlocks * 27 * WG_MAXC * 64, head_part));
    U->wg_bpart = takeF((size_t)kWgradBlocks * 64);
    U->y = takeF((size_t)U->d.out_ch * N);
    U->gy = takeF((size_t)U->d.out_ch * N);
    U->lq = takeF((size_t)U->d.out_ch * N);
    U->x0 = takeB((size_t)N * 16);
    auto act = [&](Act &a, int lvl, int ch) {
        a.n = n >> lvl;
        a.c = ch;
        a.p = takeB((size_t)a.n * a.n * a.n * ch);
    };
    const int *c = U->c;
    for (int k = 0; k < 4; ++k) act(U->ea[k], k, c[k]);
    act(U->eb3, 3, c[3]);
    for (int k = 0; k < 3; ++k) {
        act(U->cat[k], k, c[k + 1] + c[k]);
        act(U->p[k], k + 1, c[k]);
        act(U->da[k], k, c[k]);
        act(U->db[k], k, c[k]);
        act(U->g_cat[k], k, c[k + 1] + c[k]);
        act(U->g_p[k], k + 1, c[k]);
        act(U->g_da[k], k, c[k]);
        act(U->g_db[k], k, c[k]);
    }
    for (int k = 0; k < 4; ++k) act(U->g_ea[k], k, c[k]);
    act(U->g_eb3, 3, c[3]);
    act(U->g_x, 0, 16);
    return off;
}

int conv_fwd(gr_unet U, int li, const bf16 *in, int ics, int icoff, bf16 *out, int ocs, int ocoff, int n)
{
    const ConvLayer &L = U->conv[li];
    if (!launch_conv_t<true, true>(U->stream, L.cout, in, L.cin, ics, icoff, L.wf, L.kpad, U->param + L.b_off, out,
                                   ocs, ocoff, n))
        return ufail(GR_EINVAL, "unsupported channel count %d", L.cout);
    ULAUNCH();
    return GR_OK;
}

// input gradient of layer li: gin = conv(gout, flipped/transposed weights)
int conv_dgrad(gr_unet U, int li, const bf16 *gout, int gcs, int gcoff, bf16 *gin, int n)
{
    const ConvLayer &L = U->conv[li];
    if (!launch_conv_t<false, false>(U->stream, L.cin, gout, L.cout, gcs, gcoff, L.wt, L.kpadT, nullptr, gin, L.cin,
                                     0, n))
        return ufail(GR_EINVAL, "unsupported channel count %d", L.cin);
    ULAUNCH();
    return GR_OK;
}

int conv_wgrad(gr_unet U, int li, const bf16 *gout, int gcs, int gcoff, const bf16 *in, int ics, int icoff, int n)
{
    const ConvLayer &L = U->conv[li];
    const long N = (long)n * n * n;
    if (N % WG_CHUNK || L.cout % 16 || L.cin % 16 || L.cout > 64 || L.cin > WG_MAXC ||
        (L.cout / 16) * (L.cin / 16) > 4 * WG_MAXT)
        return ufail(GR_EINVAL, "weight gradient: unsupported shape (n %d, cin %d, cout %d)", n, L.cin, L.cout);
    const int nbk = (int)std::min<long>(kWgradBlocks, N / WG_CHUNK);
    k_conv3_wgrad<<<dim3((unsigned)nbk, 27), TPB, 0, U->stream>>>(gout, L.cout, gcs, gcoff, in, L.cin, ics, icoff,
                                                                 U->wg_part, U->wg_bpart, n);
    const long per = 27L * L.cout * L.cin;
    k_wgrad_reduce<<<nb(per), TPB, 0, U->stream>>>(U->wg_part, U->wg_bpart, nbk, L.cout, L.cin, U->grad + L.w_off,
                                                   U->grad + L.b_off);
    ULAUNCH();
    return GR_OK;
}

int relu_bwd(gr_unet U, bf16 *g, int gcs, int gcoff, const bf16 *a, int acs, int acoff, int c, int n)
{
    const long N = (long)n * n * n;
    k_relu_bwd<<<nb(N * c), TPB, 0, U->stream>>>(g, gcs, gcoff, a, acs, acoff, c, N);
    ULAUNCH();
    return GR_OK;
}

#define UCHK(expr)                                                                                    \
    do {                                                                                              \
        int st_ = (expr);                                                                             \
        if (st_ != GR_OK) return st_;                                                                 \
    } while (0)

int refresh_weights(gr_unet U)
{
    for (auto &L : U->conv) {
        const long tot = std::max((long)L.cout * L.kpad, (long)L.cin * L.kpadT);
        k_prep_weights<<<nb(tot), TPB, 0, U->stream>>>(U->param + L.w_off, L.cout, L.cin, L.kpad, L.kpadT, L.wf, L.wt);
    }
    ULAUNCH();
    return GR_OK;
}

// forward pass for an n^3 input (planar FP32 [in_ch][n^3]) -> U->y
int forward(gr_unet U, int n, const float *d_in)
{
    hipStream_t s = U->stream;
    const long N = (long)n * n * n;
    const int *c = U->c;
    k_pack_input<<<nb(N), TPB, 0, s>>>(d_in, U->d.in_ch, U->x0, N);
    ULAUNCH();
    // encoder
    UCHK(conv_fwd(U, E0A, U->x0, 16, 0, U->ea[0].p, c[0], 0, n));
    UCHK(conv_fwd(U, E0B, U->ea[0].p, c[0], 0, U->cat[0].p, c[1] + c[0], c[1], n));
    const bf16 *prev = nullptr;
    for (int k = 0; k < 3; ++k) {
        const int nk = n >> k, nk1 = nk >> 1;
        // pool the skip channels of cat[k]
        k_pool<<<nb((long)nk1 * nk1 * nk1 * c[k]), TPB, 0, s>>>(U->cat[k].p, c[k + 1] + c[k], c[k + 1], c[k], U->p[k].p, nk);
        ULAUNCH();
        const int la = E1A + 2 * k, lb = E1B + 2 * k;
        UCHK(conv_fwd(U, la, U->p[k].p, c[k], 0, U->ea[k + 1].p, c[k + 1], 0, nk1));
        if (k < 2) UCHK(conv_fwd(U, lb, U->ea[k + 1].p, c[k + 1], 0, U->cat[k + 1].p, c[k + 2] + c[k + 1], c[k + 2], nk1));
        else UCHK(conv_fwd(U, lb, U->ea[3].p, c[3], 0, U->eb3.p, c[3], 0, nk1));
    }
    (void)prev;
    // decoder
    for (int k = 2; k >= 0; --k) {
        const int nk = n >> k;
        const Act &src = (k == 2) ? U->eb3 : U->db[k + 1];
        k_upsample<<<nb((long)nk * nk * nk * (src.c / 8)), TPB, 0, s>>>(src.p, src.c, U->cat[k].p, c[k + 1] + c[k], nk);
        ULAUNCH();
        const int la = D2A + 2 * (2 - k), lb = D2B + 2 * (2 - k);
        UCHK(conv_fwd(U, la, U->cat[k].p, c[k + 1] + c[k], 0, U->da[k].p, c[k], 0, nk));
        UCHK(conv_fwd(U, lb, U->da[k].p, c[k], 0, U->db[k].p, c[k], 0, nk));
    }
    k_head<<<nb(N), TPB, 0, s>>>(U->db[0].p, c[0], U->param + U->head_w, U->param + U->head_b, U->y, U->d.out_ch, N);
    ULAUNCH();
    return GR_OK;
}

// backward pass (after forward and k_mse filled U->gy): accumulates U->grad
int backward(gr_unet U, int n)
{
    hipStream_t s = U->stream;
    const long N = (long)n * n * n;
    const int *c = U->c;
    {
        const int nw = U->d.out_ch * c[0], npar = nw + U->d.out_ch;
        const unsigned nblk = nb(N);
        k_head_bwd<<<nblk, TPB, 0, s>>>(U->gy, U->db[0].p, c[0], U->param + U->head_w, U->d.out_ch, U->g_db[0].p,
                                        U->wg_part, N);
        k_head_reduce<<<(unsigned)npar, TPB, 0, s>>>(U->wg_part, (int)nblk, npar, nw, U->grad + U->head_w,
                                                     U->grad + U->head_b);
        ULAUNCH();
    }
    // decoder, fine to coarse: each level's concat gradient feeds the next coarser output
    for (int k = 0; k <= 2; ++k) {
        const int nk = n >> k;
        const int la = D2A + 2 * (2 - k), lb = D2B + 2 * (2 - k);
        const int C = c[k + 1] + c[k];
        UCHK(relu_bwd(U, U->g_db[k].p, c[k], 0, U->db[k].p, c[k], 0, c[k], nk));
        UCHK(conv_wgrad(U, lb, U->g_db[k].p, c[k], 0, U->da[k].p, c[k], 0, nk));
        UCHK(conv_dgrad(U, lb, U->g_db[k].p, c[k], 0, U->g_da[k].p, nk));
        UCHK(relu_bwd(U, U->g_da[k].p, c[k], 0, U->da[k].p, c[k], 0, c[k], nk));
        UCHK(conv_wgrad(U, la, U->g_da[k].p, c[k], 0, U->cat[k].p, C, 0, nk));
        UCHK(conv_dgrad(U, la, U->g_da[k].p, c[k], 0, U->g_cat[k].p, nk));
        // upsampled channels [0, c[k+1]) -> gradient of the coarser output
        const int m = nk / 2;
        bf16 *dst = (k == 2) ? U->g_eb3.p : U->g_db[k + 1].p;
        k_upsample_bwd<<<nb((long)m * m * m * c[k + 1]), TPB, 0, s>>>(U->g_cat[k].p, C, c[k + 1], dst, nk);
        ULAUNCH();
    }
    // bottleneck
    {
        const int n3 = n >> 3;
        UCHK(relu_bwd(U, U->g_eb3.p, c[3], 0, U->eb3.p, c[3], 0, c[3], n3));
        UCHK(conv_wgrad(U, E3B, U->g_eb3.p, c[3], 0, U->ea[3].p, c[3], 0, n3));
        UCHK(conv_dgrad(U, E3B, U->g_eb3.p, c[3], 0, U->g_ea[3].p, n3));
        UCHK(relu_bwd(U, U->g_ea[3].p, c[3], 0, U->ea[3].p, c[3], 0, c[3], n3));
        UCHK(conv_wgrad(U, E3A, U->g_ea[3].p, c[3], 0, U->p[2].p, c[2], 0, n3));
        UCHK(conv_dgrad(U, E3A, U->g_ea[3].p, c[3], 0, U->g_p[2].p, n3));
    }
    // encoder, coarse to fine: skip gradient = decoder part (in g_cat) + pooling part
    for (int k = 2; k >= 0; --k) {
        const int nk = n >> k;
        const int C = c[k + 1] + c[k];
        k_pool_bwd_add<<<nb((long)nk * nk * nk * c[k]), TPB, 0, s>>>(U->g_p[k].p, c[k], U->g_cat[k].p, C, c[k + 1], nk);
        ULAUNCH();
        const int la = E0A + 2 * k, lb = E0B + 2 * k;
        UCHK(relu_bwd(U, U->g_cat[k].p, C, c[k + 1], U->cat[k].p, C, c[k + 1], c[k], nk));
        UCHK(conv_wgrad(U, lb, U->g_cat[k].p, C, c[k + 1], U->ea[k].p, c[k], 0, nk));
        UCHK(conv_dgrad(U, lb, U->g_cat[k].p, C, c[k + 1], U->g_ea[k].p, nk));
        UCHK(relu_bwd(U, U->g_ea[k].p, c[k], 0, U->ea[k].p, c[k], 0, c[k], nk));
        if (k > 0) {
            UCHK(conv_wgrad(U, la, U->g_ea[k].p, c[k], 0, U->p[k - 1].p, c[k - 1], 0, nk));
            UCHK(conv_dgrad(U, la, U->g_ea[k].p, c[k], 0, U->g_p[k - 1].p, nk));
        } else {
            UCHK(conv_wgrad(U, la, U->g_ea[0].p, c[0], 0, U->x0, 16, 0, nk));
        }
    }
    return GR_OK;
}

// forward + MSE loss + backward; loss (mean square) returned on the host
int loss_and_grad(gr_unet U, int n, const float *d_in, const float *d_target, double *h_loss)
{
    const long N = (long)n * n * n;
    k_zero_f32<<<nb(U->nparam), TPB, 0, U->stream>>>(U->grad, U->nparam);
    ULAUNCH();
    UCHK(forward(U, n, d_in));
    const long tot = (long)U->d.out_ch * N;
    const int nbk = (int)std::min<long>(1024, (tot + TPB - 1) / TPB);
    k_mse<<<nbk, TPB, 0, U->stream>>>(U->y, d_target, U->gy, tot, U->loss_partial);
    const float lam = U->d.lap_weight;
    if (lam > 0.0f) {
        k_lap_loss1<<<nbk, TPB, 0, U->stream>>>(U->y, d_target, U->lq, n, tot, U->loss_partial + 1024);
        k_lap_loss2<<<nbk, TPB, 0, U->stream>>>(U->lq, U->gy, n, tot, lam);
    }
    ULAUNCH();
    UCHK(backward(U, n));
    if (h_loss) {
        std::vector<float> part(2 * 1024, 0.0f);
        UHIP(hipMemcpyAsync(part.data(), U->loss_partial, sizeof(float) * nbk, hipMemcpyDeviceToHost, U->stream));
        if (lam > 0.0f)
            UHIP(hipMemcpyAsync(part.data() + 1024, U->loss_partial + 1024, sizeof(float) * nbk,
                                hipMemcpyDeviceToHost, U->stream));
        UHIP(hipStreamSynchronize(U->stream));
        double acc = 0.0, accl = 0.0;
        for (int i = 0; i < nbk; ++i) {
            acc += part[i];
            accl += part[1024 + i];
        }
        *h_loss = (acc + (double)lam * accl) / (double)tot;
    }
    return GR_OK;
}

int check_n(gr_unet U, int n)
{
    if (!U || !U->bound) return ufail(U ? GR_ESTATE : GR_EINVAL, "network not bound");
    if (n < 32 || n % 32 || n > U->max_n) return ufail(GR_EINVAL, "n = %d must be a multiple of 32, <= %d", n, U->max_n);
    return GR_OK;
}

} // namespace

extern "C" {

const char *gr_unet_last_error(void) { return u_err.c_str(); }

int gr_unet_create(const gr_unet_desc *d, int max_n, gr_unet *out)
{
    if (!d || !out) return ufail(GR_EINVAL, "null argument");
    *out = nullptr;
    if (d->in_ch < 1 || d->in_ch > 16 || d->out_ch < 1 || d->out_ch > 16)
        return ufail(GR_EINVAL, "in_ch and out_ch must be 1..16");
    if (!(d->lap_weight >= 0.0f) || !std::isfinite(d->lap_weight))
        return ufail(GR_EINVAL, "lap_weight must be finite and >= 0");
    if (!(d->clip_norm >= 0.0f) || !std::isfinite(d->clip_norm))
        return ufail(GR_EINVAL, "clip_norm must be finite and >= 0");
    if (d->c[0] != 16) return ufail(GR_EINVAL, "c[0] must be 16");
    for (int k = 1; k < 4; ++k)
        if (d->c[k] < 16 || d->c[k] > 64 || d->c[k] % 16) return ufail(GR_EINVAL, "c[%d] must be 16, 32, 48 or 64", k);
    if (max_n < 32 || max_n % 32 || max_n > 512) return ufail(GR_EINVAL, "max_n must be a multiple of 32 up to 512");
    gr_unet U = new (std::nothrow) gr_unet_s();
    if (!U) return ufail(GR_EINVAL, "out of host memory");
    U->d = *d;
    U->max_n = max_n;
    for (int k = 0; k < 4; ++k) U->c[k] = d->c[k];
    const int *c = U->c;
    const int io[14][2] = {{16, c[0]}, {c[0], c[0]}, {c[0], c[1]}, {c[1], c[1]}, {c[1], c[2]}, {c[2], c[2]},
                           {c[2], c[3]}, {c[3], c[3]}, {c[3] + c[2], c[2]}, {c[2], c[2]}, {c[2] + c[1], c[1]},
                           {c[1], c[1]}, {c[1] + c[0], c[0]}, {c[0], c[0]}};
    long off = 0;
    for (int l = 0; l < 14; ++l) {
        ConvLayer &L = U->conv[l];
        L.cin = io[l][0];
        L.cout = io[l][1];
        L.kpad = pad32(27 * L.cin);
        L.kpadT = pad32(27 * L.cout);
        L.w_off = off;
        off += (long)L.cout * 27 * L.cin;
        L.b_off = off;
        off += L.cout;
    }
    U->head_w = off;
    off += (long)d->out_ch * c[0];
    U->head_b = off;
    off += d->out_ch;
    U->nparam = off;
    U->ws_bytes = unet_layout(U, nullptr);
    *out = U;
    return GR_OK;
}

int gr_unet_workspace_bytes(gr_unet U, size_t *bytes)
{
    if (!U || !bytes) return ufail(GR_EINVAL, "null argument");
    *bytes = U->ws_bytes;
    return GR_OK;
}

int gr_unet_param_count(gr_unet U, int64_t *count)
{
    if (!U || !count) return ufail(GR_EINVAL, "null argument");
    *count = U->nparam;
    return GR_OK;
}

int gr_unet_bind(gr_unet U, void *d_ws, size_t bytes, void *stream)
{
    if (!U || !d_ws) return ufail(GR_EINVAL, "null argument");
    if (bytes < U->ws_bytes) return ufail(GR_EINVAL, "workspace %zu bytes < required %zu", bytes, U->ws_bytes);
    if (reinterpret_cast<uintptr_t>(d_ws) % 256) return ufail(GR_EINVAL, "workspace not 256-byte aligned");
    U->stream = reinterpret_cast<hipStream_t>(stream);
    unet_layout(U, reinterpret_cast<char *>(d_ws));
    const long nw = (long)(U->ws_bytes / sizeof(float));
    k_zero_f32<<<nb(nw), TPB, 0, U->stream>>>(reinterpret_cast<float *>(d_ws), nw);
    ULAUNCH();
    U->bound = true;
    U->step = 0;
    return GR_OK;
}

// He-normal weights (std sqrt(2 / fan_in)), zero biases, zero Adam moments.
int gr_unet_init(gr_unet U, uint64_t seed)
{
    if (!U || !U->bound) return ufail(U ? GR_ESTATE : GR_EINVAL, "network not bound");
    hipStream_t s = U->stream;
    k_zero_f32<<<nb(U->nparam), TPB, 0, s>>>(U->param, U->nparam);
    k_zero_f32<<<nb(U->nparam), TPB, 0, s>>>(U->adam_m, U->nparam);
    k_zero_f32<<<nb(U->nparam), TPB, 0, s>>>(U->adam_v, U->nparam);
    for (int l = 0; l < 14; ++l) {
        const ConvLayer &L = U->conv[l];
        const long cnt = (long)L.cout * 27 * L.cin;
        k_init_normal<<<nb(cnt), TPB, 0, s>>>(U->param + L.w_off, cnt, std::sqrt(2.0f / (27.0f * L.cin)),
                                             seed * 1000003ull + l);
    }
    const long hc = (long)U->d.out_ch * U->c[0];
    k_init_normal<<<nb(hc), TPB, 0, s>>>(U->param + U->head_w, hc, std::sqrt(1.0f / U->c[0]), seed * 1000003ull + 99);
    ULAUNCH();
    U->step = 0;
    return refresh_weights(U);
}

int gr_unet_set_params(gr_unet U, const float *d_src)
{
    if (!U || !U->bound || !d_src) return ufail(GR_EINVAL, "bad argument");
    UHIP(hipMemcpyAsync(U->param, d_src, sizeof(float) * U->nparam, hipMemcpyDeviceToDevice, U->stream));
    return refresh_weights(U);
}

int gr_unet_get_params(gr_unet U, float *d_dst)
{
    if (!U || !U->bound || !d_dst) return ufail(GR_EINVAL, "bad argument");
    UHIP(hipMemcpyAsync(d_dst, U->param, sizeof(float) * U->nparam, hipMemcpyDeviceToDevice, U->stream));
    return GR_OK;
}

int gr_unet_forward(gr_unet U, int n, const float *d_in, float *d_out)
{
    int st = check_n(U, n);
    if (st) return st;
    if (!d_in || !d_out) return ufail(GR_EINVAL, "null tensor");
    UCHK(forward(U, n, d_in));
    const long N = (long)n * n * n;
    UHIP(hipMemcpyAsync(d_out, U->y, sizeof(float) * U->d.out_ch * N, hipMemcpyDeviceToDevice, U->stream));
    return GR_OK;
}

int gr_unet_loss_grad(gr_unet U, int n, const float *d_in, const float *d_target, float *d_grad, double *h_loss)
{
    int st = check_n(U, n);
    if (st) return st;
    if (!d_in || !d_target) return ufail(GR_EINVAL, "null tensor");
    UCHK(loss_and_grad(U, n, d_in, d_target, h_loss));
    if (d_grad)
        UHIP(hipMemcpyAsync(d_grad, U->grad, sizeof(float) * U->nparam, hipMemcpyDeviceToDevice, U->stream));
    return GR_OK;
}

int gr_unet_train_step(gr_unet U, int n, const float *d_in, const float *d_target, float lr, double *h_loss)
{
    int st = check_n(U, n);
    if (st) return st;
    if (!d_in || !d_target || !(lr > 0.0f)) return ufail(GR_EINVAL, "bad argument");
    UCHK(loss_and_grad(U, n, d_in, d_target, h_loss));
    ++U->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float clip = U->d.clip_norm > 0.0f ? U->d.clip_norm : 3.4e38f;
    k_sumsq<<<kClipBlocks, TPB, 0, U->stream>>>(U->grad, U->nparam, U->gn_part);
    k_clip_scale<<<1, 64, 0, U->stream>>>(U->gn_part, kClipBlocks, clip, U->gscale, U->gscale + 1);
    k_adam<<<nb(U->nparam), TPB, 0, U->stream>>>(U->param, U->grad, U->adam_m, U->adam_v, U->nparam, lr, b1, b2, 1e-8f,
                                                1.0f - std::pow(b1, (float)U->step), 1.0f - std::pow(b2, (float)U->step),
                                                U->gscale);
    ULAUNCH();
    return refresh_weights(U);
}

int gr_destroy_unet(gr_unet U)
{
    delete U;
    return GR_OK;
}

} // extern "C"
