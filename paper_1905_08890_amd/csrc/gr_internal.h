// Internal declarations shared by the HIP translation units of libgrmg.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gr.h"

namespace grmg {

constexpr int kMaxLevels = 12;
constexpr int kCoarseSweeps = 32;   // red-black sweeps at the coarsest level
constexpr int kReduceBlocks = 4096; // partial-sum slots per reduction (the grid for a size is fixed => deterministic)
constexpr int kReduceThreads = 256;

// Device scalar slots (doubles) in the workspace.
enum Slot {
    S_ZERO = 0,      // always 0: frozen scalars of coarse levels
    S_MEAN = 1,      // mean for pinning / correction projection
    S_FBAR = 2,      // Hamiltonian regulariser <F> (finest level)
    S_FSHIFT = 3,    // CMC finest-level source shift <f> + <m2 xi>
    S_FMEAN = 4,     // CMC <f> (once per solve)
    S_RN = 5,        // sum eps^2   (pair with S_FN)
    S_FN = 6,        // sum (f - fshift)^2
    S_SCRATCH = 8,   // 8 general slots
    S_NUM = 32
};

// FP32 arrays of one level for the correction cycles: correction e, its
// source b, coefficients a (Hamiltonian: chi) and c, and a scratch buffer.
struct Level32 {
    float *e, *b, *a, *c, *tmp;
};

// Linearised (correction) operators J e = a Lap e + c e of the three kinds,
// used in FP32 by the inner cycles of mixed-precision refinement.
constexpr int K_LIN_POISSON = 3, K_LIN_HAM = 4, K_LIN_CMC = 5;

// Operator constants of one equation.
struct OpConst {
    double kappa; // 1/(2 a^2 c^2)
    double A;     // 3/2 a Om
};

struct Level {
    int n;
    double h;
    long N;
    double *phi;  // level iterate (level 0: the field itself, set per solve)
    double *phi0; // restricted iterate R phi (FAS), or saved copy at the coarsest
    double *f;    // level source (level 0: fine source GR_RHS)
    double *coef; // operator coefficient (level 0: GR_COEF)
    double *tmp;  // scratch of the level size
};


// ---- stencil.hip launchers ----
void launch_rb_sweep(int kind, hipStream_t s, double *phi, const double *f, const double *coef, int n,
                     double h, OpConst oc, const double *fbar, const double *fshift);
// fused out-of-place sweep (both colours, one pass); used where fused_sweep_ok
struct FusedCfg {
    int min_n = 128;      // smallest level that uses it (smaller levels: one kernel per colour)
    int tile = 2;         // 0: 64x8 tiles, 1: 32x16, 2: 64x16, 3: 128x8 (n % 128 == 0)
    int xcd_remap = 2;    // 0: z-chunk fastest, 1: XCD-contiguous workgroup order, 2: XCD-contiguous tile regions
    int target_wgs = 256; // about one workgroup per CU (measured best for the FP64 kinds at 256^3)
    int pf = 0;           // operand prefetch depth in planes (1 or 2; 0: per-kind default)
};
bool fused_sweep_ok(int n, int min_n);
void launch_rb_fused(int kind, hipStream_t s, const double *in, double *out, const double *f, const double *coef,
                     int n, double h, OpConst oc, const double *fbar, const double *fshift, const FusedCfg &cfg);
// The whole V-cycle from a small level down, in one single-workgroup launch.
// FAS kinds: phi/phi0/f/c1 = iterate, R phi, source, coefficient.  Linearised
// kinds: phi = correction e, f = its source b, c1 = c, c2 = a.
template <typename T> struct CoarseLevelsT {
    int nl;                    // levels held (first = the level the cycle starts on)
    int n[kMaxLevels];
    double inv_h2[kMaxLevels];
    T *phi[kMaxLevels], *phi0[kMaxLevels], *f[kMaxLevels], *c1[kMaxLevels], *c2[kMaxLevels], *tmp[kMaxLevels];
};
void launch_coarse_vcycle(int kind, hipStream_t s, const CoarseLevelsT<double> &C, int nu1, int nu2, OpConst oc,
                          const double *fbar0, const double *fshift0);
void launch_coarse_vcycle_f32(int kind, hipStream_t s, const CoarseLevelsT<float> &C, int nu1, int nu2, OpConst oc,
                              const double *zero);

// ---- FP32 correction-scheme kernels (mixed precision) ----
void launch_rb_sweep_f32(int kind, hipStream_t s, float *e, const float *b, const float *c1, const float *c2, int n,
                         double h, OpConst oc, const double *zero);
void launch_rb_fused_f32(int kind, hipStream_t s, const float *in, float *out, const float *b, const float *c1,
                         const float *c2, int n, double h, OpConst oc, const double *zero, const FusedCfg &cfg);
void launch_lin_residual_restrict_f32(int kind, hipStream_t s, const float *e, const float *b, const float *c1,
                                      const float *c2, int n, double h, OpConst oc, float *b_c, float *e_c);
void launch_prolong_add_f32(hipStream_t s, float *e_f, int n, const float *e_c);
void launch_prolong_add_f64(hipStream_t s, double *phi_f, int n, const double *e_c);
void launch_sub_arrays(hipStream_t s, double *d, const double *a, const double *b, long N);
void launch_ir_update_residual(hipStream_t s, const double *phi, const float *e, double *phi_out, const double *f,
                               int n, double h, OpConst oc, const double *fbar, const double *fshift, float *b32,
                               double *partials);
void launch_restrict_f32(hipStream_t s, const float *fine, int n, float *coarse);
void launch_ir_residual(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                        double h, OpConst oc, const double *fbar, const double *fshift, float *b32, float *a32,
                        float *c32, double *partials);
void launch_neg_to_f32(hipStream_t s, float *dst, const double *src, long N);
void launch_sum_f32(hipStream_t s, const float *x, long N, double *partials);
void launch_ir_update(hipStream_t s, double *phi, const float *e, long N, const double *mean);
// phi += e - <e>, fused with the next pass's sum over phi: of F (Hamiltonian;
// coef = AA) or of coef * phi (CMC; coef = m2), partial sums as launch_sum_ham_F /
// launch_sum_prod
void launch_ir_update_sum(int kind, hipStream_t s, double *phi, const float *e, const double *mean, const double *f,
                          const double *coef, long N, OpConst oc, double *partials);
// the FP32 linearisation arrays a and c restricted one level (n: fine side)
void launch_restrict2_f32(hipStream_t s, const float *fa, const float *fc, int n, float *ca, float *cc);
// the same through levels 0..nl (sides n[0], n[0]/2, ...) in one workgroup
struct RestrictChain {
    int nl; // restrictions done: level l -> l + 1 for l < nl
    int n[kMaxLevels];
    float *a[kMaxLevels], *c[kMaxLevels];
};
void launch_restrict2_chain(hipStream_t s, const RestrictChain &R);
void launch_fill_f32(hipStream_t s, float *x, long N);
void launch_copy_f32(hipStream_t s, float *dst, const float *src, long N);

void launch_residual_restrict(int kind, hipStream_t s, const double *phi, const double *f,
                              const double *coef, int n, double h, OpConst oc, const double *fbar,
                              const double *fshift, double *phi_c, double *phi0_c, double *rr_c);
void launch_coarse_rhs(int kind, hipStream_t s, const double *phi_c, const double *coef_c,
                       const double *rr_c, int m, double H, OpConst oc, double *f_c);
void launch_prolong_correct(hipStream_t s, double *phi_f, int n, const double *phi_c, const double *phi0_c);
void launch_restrict(hipStream_t s, const double *fine, int n, double *coarse);
void launch_residual(int kind, hipStream_t s, const double *phi, const double *f, const double *coef, int n,
                     double h, OpConst oc, const double *fbar, const double *fshift, double *r);

// reductions: partial sums (kReduceBlocks x ncomp) then a fixed-order finalise
// out[slot + c] = add[c] + scale * sum_c   (add may be null)
void launch_sum(hipStream_t s, const double *x, const double *y, long N, double *partials);
void launch_sum_ham_F(hipStream_t s, const double *psi, const double *f, const double *coef, long N,
                      OpConst oc, double *partials);
void launch_sum_prod(hipStream_t s, const double *x, const double *y, long N, double *partials);
void launch_res_norms(int kind, hipStream_t s, const double *phi, const double *f, const double *coef,
                      int n, double h, OpConst oc, const double *fbar, const double *fshift,
                      double *partials);
// out[c] = add[c] + scale * (fixed-order sum of the partials of quantity c);
// host_out (optional): page-locked, coherent host memory that receives the same
// values, written before the kernel ends (the per-cycle stopping norms)
void launch_finalize(hipStream_t s, const double *partials, int ncomp, double scale, const double *add,
                     double *out, double *host_out = nullptr);

void launch_fill(hipStream_t s, double *x, long N, double v);
void launch_copy(hipStream_t s, double *dst, const double *src, long N);
void launch_sub_scalar(hipStream_t s, double *x, long N, const double *scal);
void launch_convert_f32_to_f64(hipStream_t s, double *dst, const float *src, long N);
void launch_convert_f64_to_f32(hipStream_t s, float *dst, const double *src, long N);
void launch_set_scalar(hipStream_t s, double *slot, double v);
void launch_affine_to_f32(hipStream_t s, float *dst, const double *src, long N, double off, double scale, bool acc);
void launch_f32_scaled_to_f64(hipStream_t s, double *dst, const float *src, long N, double scale);
void launch_axpy(hipStream_t s, double *y, const double *x, long N);
// field, history, alternative: old = field; alt = old; field = (hv ? 2 old - hist : old) + add; hist = old
void launch_extrapolate(hipStream_t s, double *field, double *hist, double *alt, const double *add, bool hv, long N);
void launch_cubic_pass(hipStream_t s, const double *in, int nx, int ny, int nz, int dim, double *out);

// ---- sources.hip launchers ----
// cell-ordered deposit for up to `cap` particles; scratch of cic_sorted_bytes(N, cap)
size_t cic_sorted_bytes(long N, long cap);
void launch_cic_sorted(hipStream_t s, int n, double a, double c_tilde, const double *pos, const double *u,
                       double mass, long np, const double *psi, void *scratch, double *s0, double *sx, double *sy,
                       double *sz, double *sm);
void launch_cic_deposit(hipStream_t s, int n, double a, double c_tilde, const double *pos, const double *u,
                        double mass, long np, const double *psi, double *s0, double *sx, double *sy,
                        double *sz, double *sm);
void launch_shift_scale(hipStream_t s, double *out, const double *in, long N, double scale,
                        const double *mean);
void launch_div_quarter(hipStream_t s, double *out, const double *gx, const double *gy, const double *gz,
                        int n, double h);
void launch_build_Aij(hipStream_t s, double *const A6[6], double *AA, const double *Vx, const double *Vy,
                      const double *Vz, const double *U, int n, double h);
void launch_ham_rhs(hipStream_t s, double *f, const double *s0, long N, double A);
void launch_build_cmc(hipStream_t s, double *m2, double *f, const double *psi, const double *s0,
                      const double *sm, const double *AA, long N, double a, double om, double c_tilde);
void launch_shift_source(hipStream_t s, double *fB[3], const double *psi, const double *xi,
                         double *const A6[6], int n, double h, double a, double c_tilde);
// ---- particles.hip launchers (fields: Phi, Psi and beta^i grids of side n) ----
void launch_kick(hipStream_t s, int n, double a, double c, const double *Phi, const double *Psi,
                 const double *const beta[3], const double *pos, double *u, long np, double dt, int order);
void launch_newton_kick(hipStream_t s, int n, const double *phiN, const double *pos, double *u, long np, double dt);
void launch_drift(hipStream_t s, int n, double a, double c, const double *Phi, const double *Psi,
                  const double *const beta[3], double *pos, const double *u, long np, double dt);
void launch_derived(hipStream_t s, int which, double *out, const double *psi, const double *xi,
                    const double *Bcomp, const double *b, int n, double h, double a, double c_tilde);

} // namespace grmg
