/*
 * gr.h - C ABI of the MI355X (gfx950) constraint/gauge solver for the
 * constrained-ADM N-body method of Barrera-Hinojosa & Li 2019 ("GRAMSES I").
 *
 * Every time step the method solves, on a periodic box in conformal flatness,
 * ten elliptic equations (paper sec. 2.4 solution scheme, code-unit forms of
 * sec. 4.1.1, multigrid forms of sec. 4.3):
 *   V_i  : Lap V_i = 3 Om a (s_i - <s_i>)                 (momentum constraint)
 *   U    : Lap U   = -1/4 d_j V^j
 *   Psi  : regularised Hamiltonian constraint, chi = 1 - Psi/(2 a^2 c^2),
 *          psi = a^(1/2) chi                               (sec. 4.3.2.1)
 *   xi   : regularised CMC lapse equation, xi = Phi chi, alpha = 1 + Phi/(a^2c^2)
 *                                                          (sec. 4.3.2.2)
 *   B^i  : Lap B^i = 2 d_j[alpha chi^-6 A^ij]              (shift, MD gauge)
 *   b    : Lap b   = -1/4 d_j B^j,  beta^i = B^i + d^i b
 * with A_ij = d_iV_j + d_jV_i - 1/2 delta_ij d_kV^k + 2 d_i d_j U, all on a
 * cell-centred uniform grid with the 7-point Laplacian and 3-point central
 * differences of sec. 4.3.1, by FAS multigrid V-cycles smoothed by red-black
 * Gauss-Seidel with one pointwise Newton step per visit.
 *
 * Conventions
 *   - Every function returns an int status: GR_OK (0) or a negative code;
 *     gr_last_error() gives a thread-local message.  No C++ exception crosses
 *     the ABI.
 *   - Device memory belongs to the caller.  gr_workspace_bytes() says how much
 *     one grid needs; the caller allocates it (e.g. a torch uint8 tensor) and
 *     hands it over with gr_bind().  After gr_bind() the library never
 *     allocates device memory (gr_bind itself creates the grid's private
 *     streams and events and 16 bytes of pinned host memory per hierarchy for
 *     the per-cycle norm read-back).  The workspace must outlive the handle.
 *   - Arrays are float64 (or float32 where a dtype argument says so),
 *     C order [z][y][x] with x fastest, n^3 elements, device pointers.
 *   - All work is enqueued on the stream given to gr_bind() (a hipStream_t;
 *     NULL = the null stream).  Calls are stream-ordered; only
 *     gr_solve_constraints() and gr_solve_equation() synchronise the stream,
 *     once per V-cycle, to read the 16-byte residual norm that decides
 *     stopping, and before returning.
 *   - Handles are not thread-safe: one thread at a time per grid.
 */
#ifndef GR_H
#define GR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define GR_OK 0
#define GR_EINVAL (-1)    /* bad argument: null pointer, size, field id, dtype   */
#define GR_EDEVICE (-2)   /* a HIP call failed                                   */
#define GR_ENOTCONV (-3)  /* max_cycles reached before rtol (report is filled)   */
#define GR_ENAN (-4)      /* NaN/Inf in a residual norm (report is filled)       */
#define GR_ESTATE (-6)    /* grid not bound to a workspace                       */

/* ---- equation kinds (low-level gr_solve_equation) ---- */
#define GR_KIND_POISSON 0     /* Lap phi = f                                     */
#define GR_KIND_HAMILTONIAN 1 /* chi Lap Psi + A(chi^6-1) - AA chi^-6/4 + <F>chi = f */
#define GR_KIND_CMC 2         /* Lap xi - m2 xi = f - <f> - <m2 xi>              */

/* ---- field ids ---- */
enum {
    /* the ten solved potentials, in solve order groups */
    GR_VX = 0, GR_VY = 1, GR_VZ = 2, GR_U = 3, GR_PSI = 4, GR_XI = 5,
    GR_BX = 6, GR_BY = 7, GR_BZ = 8, GR_BB = 9,
    /* matter sources (conformal, code units; sec. 3 and 4.1.2) */
    GR_S0 = 10, GR_SX = 11, GR_SY = 12, GR_SZ = 13, GR_SM = 14,
    /* geometric source A_ij A^ij, valid after a solve that built it */
    GR_AA = 15,
    /* derived, get only: Phi = xi/chi, alpha = 1 + Phi/(a^2c^2),
       psi = a^(1/2) chi, beta^i = B^i + d_i b */
    GR_PHI = 16, GR_ALPHA = 17, GR_CONF = 18, GR_BETAX = 19, GR_BETAY = 20, GR_BETAZ = 21,
    /* low-level slots read by gr_solve_equation / gr_debug_*: fine source f
       and operator coefficient (AA for the Hamiltonian, m2 for CMC) */
    GR_RHS = 22, GR_COEF = 23,
    /* solved field f's history (GR_HIST + f): its value before the last
       gr_set_guess with GR_SET_EXTRAP; gr_set_field on it sets the history
       and marks it recorded, a gr_solve_constraints from GR_GUESS_ZERO
       discards it (a new trajectory) */
    GR_HIST = 24,
    GR_NUM_FIELD_IDS = 34
};

#define GR_F64 0
#define GR_F32 1

#define GR_FP64 0   /* plain FP64 multigrid                                   */
#define GR_MIXED 1  /* FP32 inner V-cycles, FP64 residual/update (iterative refinement) */

#define GR_GUESS_ZERO 0     /* start every solved field from 0                 */
#define GR_GUESS_CURRENT 1  /* start from the values held (previous step / set_field) */
#define GR_GUESS_CHECKED 2  /* as CURRENT, but per field take the saved alternative
                               (previous-step values saved by gr_set_guess) unless the
                               held guess has the strictly smaller FP64 residual (a
                               non-finite held guess never does); ties take the
                               alternative.  Any solve of a field uses up its saved
                               alternative. */

#define GR_ALL_FIELDS 0x3FFu

typedef struct gr_grid_s *gr_grid;

/* Code-unit parameters (sec. 4.1.1): fiducial scale factor a, Omega_m and the
 * speed of light c~ = c/(L H0). */
typedef struct {
    double a;
    double omega_m;
    double c_tilde;
} gr_params;

/* Periodic cube of n^3 cells of spacing h (h = 1/n for the unit box).
 * n must be even and >= 2; the multigrid hierarchy halves n while n/2 is
 * even (so 2^k grids go down to 2^3, 48 and 96 down to 6^3). */
typedef struct {
    int n;
    double h;
} gr_grid_desc;

/* Solve options.  Defaults (what a zeroed struct means is NOT the default;
 * use gr_default_opts): nu1 = nu2 = 2, max_cycles = 100, rtol = 1e-10,
 * precision = GR_FP64, guess = GR_GUESS_ZERO, field_mask = GR_ALL_FIELDS.
 * Stopping: at the start of each cycle, rms(eps)/rms(f) <= rtol with eps the
 * fine residual L(phi) - f of the (regularised) equation (a zero source uses
 * rms(eps) <= rtol).  rtol <= 0 runs exactly max_cycles cycles and
 * returns GR_OK. */
typedef struct {
    int nu1, nu2, max_cycles;
    double rtol;
    int precision;
    int guess;
    unsigned field_mask;
} gr_solve_opts;

typedef struct {
    int status;
    int cycles[10];     /* V-cycles (mixed: refinement steps) per field        */
    double rel_res[10]; /* final rms(eps)/rms(f) per field                     */
    double seconds;     /* host wall time of the call                          */
    int fallback;       /* mixed precision: fields that fell back to FP64      */
    int guess_fallback; /* GR_GUESS_CHECKED: fields that used the alternative   */
    double guess_rel[10]; /* GR_GUESS_CHECKED: stopping quantity of the held guess  */
    double alt_rel[10];   /* ... and of the saved alternative (both 0 when none)    */
} gr_solve_report;

/* Fill *o with the defaults above. */
int gr_default_opts(gr_solve_opts *o);

/* Create a grid handle (host memory only).  Errors: GR_EINVAL for a null
 * pointer, odd or < 2 n, n > 1024, h <= 0, or non-positive a / c~. */
int gr_create_grid(const gr_grid_desc *desc, const gr_params *prm, gr_grid *out);

/* Bytes of device workspace the grid needs (all levels, all fields). */
int gr_workspace_bytes(gr_grid g, size_t *bytes);

/* Bind caller-owned device memory (>= gr_workspace_bytes, 256-byte aligned)
 * and a hipStream_t (may be NULL).  Zero-fills every field and source.
 * Re-binding replaces both. */
int gr_bind(gr_grid g, void *d_workspace, size_t bytes, void *hip_stream);

/* CIC deposit of the conformal matter sources (sec. 4.1.2) from np particles:
 * d_pos[np][3] positions in [0,1) (x,y,z), d_u[np][3] lower-index momenta u_i,
 * equal masses `mass` (code units).  Cell-centred cloud-in-cell weights with
 * periodic wrap; the Lorentz factor W^2 = c^2 + a^-2 chi^-4 u_i u_i uses the
 * Psi currently held (the previous step's Psi^n, sec. 4.5), CIC-interpolated
 * to the particle.  Overwrites s0, s_i and the stress trace s_m
 * (s_m = gamma^ij s_ij += w m a^-2 chi^-4 u_i u_i/(W c h^3)).  Positions
 * outside [0,1) are wrapped.  Up to n^3 particles are deposited in cell order
 * (counting sort by cloud corner, then one sum per grid point, no
 * floating-point atomics); more particles fall back to an atomic scatter. */
int gr_deposit_sources(gr_grid g, const double *d_pos, const double *d_u, double mass,
                       int64_t n_particles);

/* Particle evolution with the metric the grid holds (its last solve), sec. 4.4
 * and the leapfrog of the appendix on time evolution.  The metric at a
 * particle is the cloud-in-cell interpolation (the deposit's cell-centred
 * weights, periodic) of Phi = xi/chi, Psi, beta^i = B^i + d_i b and of their
 * 3-point central-difference gradients; W^2 = c^2 + a^-2 chi^-4 u.u from the
 * interpolated Psi and the particle's current u (lower-index, code units).
 * gr_kick: u_i += dt sum_j c_j (f_j)_i in five substeps, each taking c_j from
 * the velocity as updated by the substeps before it:
 *   j = 1, 2, 3: c_j = -u_j, (f_j)_i = -d_i beta^j;
 *   j = 4: c_4 = (W^2 - c^2)/(W c) (1 + Phi/(a^2c^2))/(1 - Psi/(2a^2c^2)), (f_4)_i = -d_i Psi;
 *   j = 5: c_5 = W/c, (f_5)_i = -d_i Phi;
 * order GR_KICK_FORWARD runs j = 1..5 (the synchronising kick, dominant term
 * last), GR_KICK_REVERSE j = 5..1 (the first kick); dt is the kick's length
 * (dt/2 of a time step for a half kick).
 * gr_drift: x^i += dt [(1 + Phi/(a^2c^2)) chi^-4 (c/W) u_i - beta^i] with the
 * metric at the old position, positions wrapped into [0, 1).
 * d_pos, d_u: [np][3] float64 device arrays (the caller's).  Both run on the
 * grid's stream without synchronising and use the grid's A_ij scratch for Phi
 * and beta (rebuilt by the next solve).  Errors: GR_ESTATE if unbound,
 * GR_EINVAL for null arrays with np > 0, np < 0, non-finite dt, a bad order,
 * or a grid that is not the unit box (h != 1/n). */
#define GR_KICK_FORWARD 0
#define GR_KICK_REVERSE 1
int gr_kick(gr_grid g, const double *d_pos, double *d_u, int64_t n_particles, double dt, int order);
int gr_drift(gr_grid g, double *d_pos, const double *d_u, int64_t n_particles, double dt);

/* The Newtonian half of the temporary synchronisation option (sec. 4.5, last
 * paragraph; appendix on time evolution): solves the code-unit Newtonian
 * Poisson equation Lap Phi_N = 3/2 a Om (s0 - <s0>) from the held s0 (Poisson
 * V-cycles from zero with opts' rtol, max_cycles and precision; zero mean),
 * then u_i -= dt d_i Phi_N at every particle (the same interpolation as
 * gr_kick).  With dt = half a time step this gives u_N^{n+1} from u^{n+1/2};
 * the caller keeps a copy of u to revert to exactly after depositing with u_N
 * and solving.  Fills cycles[0] / rel_res[0] of the report; synchronises the
 * stream before returning.  Uses the grid's A_ij scratch for Phi_N.  Errors as
 * gr_kick, plus bad options (GR_GUESS_CHECKED is rejected). */
int gr_newtonian_kick(gr_grid g, const double *d_pos, double *d_u, int64_t n_particles, double dt,
                      const gr_solve_opts *opts, gr_solve_report *host_report);

/* Copy n^3 values of dtype GR_F64/GR_F32 from d_src into a field slot
 * (solved fields as guesses, sources, GR_RHS, GR_COEF).  Derived ids are
 * rejected with GR_EINVAL. */
int gr_set_field(gr_grid g, int field, const void *d_src, int dtype);

/* Copy (or, for derived ids, compute) a field into d_dst (n^3 of dtype). */
int gr_get_field(gr_grid g, int field, void *d_dst, int dtype);

/* Solve the ten equations in the order V_i -> U -> (A_ij, AA) -> Psi -> xi ->
 * B^i -> b from the sources held (sec. 2.4 steps 1-4; sec. 4.3 forms).
 * Fields outside opts->field_mask are not solved; their held values feed
 * later equations.  host_report may be NULL.  Returns the first non-OK
 * status among the fields (all fields are still attempted). */
int gr_solve_constraints(gr_grid g, const gr_solve_opts *opts, gr_solve_report *host_report);

/* Low level: solve one equation of `kind` for field slot `field` (0..9) with
 * source GR_RHS and coefficient GR_COEF as set by gr_set_field.  Fills
 * cycles[0] / rel_res[0] of the report. */
int gr_solve_equation(gr_grid g, int kind, int field, const gr_solve_opts *opts,
                      gr_solve_report *host_report);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, serving loops, harnesses that forbid allocation): the solve of
 * gr_solve_equation without a grid handle or workspace.  Solves one equation
 * of `kind` on the periodic unit box of n^3 cells (h = 1/n) for d_phi, with
 * fine source d_f and coefficient d_coef (A_ijA^ij for the Hamiltonian, m^2
 * for CMC; ignored, may be NULL, for Poisson), all n^3 float64 device arrays
 * owned by the caller (d_phi: guess in with GR_GUESS_CURRENT, solution out).
 * Same equations, readings, kernels and results as gr_solve_equation on a grid
 * of side n (one-launch-per-colour smoothing, the library's default launch
 * shapes, no graph replay), enqueued on hip_stream (NULL = null stream),
 * synchronising it once per cycle and before returning.  Fills cycles[0],
 * rel_res[0] and fallback of the report.
 * Device memory: none is allocated.  The level hierarchy lives in a static
 * 16 MiB device array of the library (one per GPU, held until the process
 * ends), which limits n to even values from 2 to 64; larger n, odd n, a
 * missing coefficient, GR_GUESS_CHECKED or bad options give GR_EINVAL.  Every
 * call on a GPU shares that GPU's array, clears it at its start and leaves
 * its contents behind; calls from several host threads of one process are
 * serialised by a lock (overlapping calls would otherwise race on the array). */
int gr_solve_equation_static(int n, const gr_params *prm, int kind, const double *d_f, const double *d_coef,
                             double *d_phi, const gr_solve_opts *opts, void *hip_stream, gr_solve_report *rep);

/* Learned-guess support (the network itself is gr_unet_*).  gr_features: for
 * each of `count` field ids (solved fields, sources, GR_AA), restrict it to
 * multigrid level `level` (mean of the 8 children, applied level by level;
 * level 0 = the grid itself) and write (value - offset[c]) * scale[c] as FP32
 * to d_dst[c][n_level^3]; with GR_FEAT_ACCUMULATE in flags the value is added
 * to what d_dst holds (e.g. a snapshot taken with scale -1 before a deposit
 * gives the change of a source).
 * gr_set_guess: for each of `count` solved fields, take d_src[c][n_level^3]
 * times scale[c] and bring it to the finest level, level by level, with the
 * multigrid prolongation (cell-centred trilinear) or, with GR_SET_CUBIC in
 * flags, with 4-point Lagrange cubic interpolation per dimension (its
 * discrete Laplacian shows far smaller interpolation kinks).  With GR_SET_ADD it
 * is added to the held field after the held values are saved as that field's
 * alternative guess (see GR_GUESS_CHECKED); without, it replaces the field
 * (and clears the alternative).  With GR_SET_EXTRAP (for trajectories of time
 * steps) the held field f (the previous step) is first extrapolated linearly
 * from its history h (the step before, see GR_HIST): the field becomes
 * (2 f - h) + prediction, or f + prediction when no history has been recorded
 * yet; f is then saved both as the alternative and as the new history.  A
 * zero scale gives the plain linear extrapolation.
 * Both run on the grid's stream, read and write device memory only, and
 * return GR_EINVAL for a bad level, count, field id, flag or null pointer
 * (nothing is launched then).  d_dst / d_src hold count * n_level^3 floats,
 * owned by the caller. */
#define GR_SET_ADD 1
#define GR_SET_CUBIC 2
#define GR_SET_EXTRAP 4
#define GR_FEAT_ACCUMULATE 1
int gr_features(gr_grid g, int level, int count, const int *fields, const double *offset, const double *scale,
                float *d_dst, int flags);
int gr_set_guess(gr_grid g, int level, int count, const int *fields, const double *scale, const float *d_src,
                 int flags);

/* Autotuner of the fused red-black sweep (sec. 4.3.1 smoother): for every
 * level the fused sweep can tile (n >= 32, n % 32 == 0) and each of the six
 * operator kinds (FP64 Poisson, Hamiltonian, CMC; their FP32 linearised
 * forms), times every candidate launch configuration on workspace scratch:
 * tile 64x8, 32x16, 64x16 or (n % 128 == 0) 128x8 (only 32x16 where n % 64 ==
 * 32); a target of 256, 512,
 * 1024 or 2048 workgroups; operand prefetch 1 or 2 planes (1 to 4 for the
 * 64x16 tile); and one launch per colour instead of the fused sweep.  It
 * keeps the fastest for this grid; results are cached per process by
 * (n, kind).  Results of the sweeps
 * do not depend on the configuration.  Writes one line per (level, kind) to
 * report (may be NULL).  Must not overlap a deposit on the same grid (it uses
 * the deposit's scratch).  Errors: GR_ESTATE if unbound, GR_EDEVICE. */
int gr_autotune(gr_grid g, char *report, size_t report_bytes);

/* Timing of the finest-level fused sweeps (measurement support): with
 * enable != 0, later solves bracket every finest-level fused sweep launch with
 * HIP events on the solve's stream (cycle graphs are off meanwhile);
 * enable == 0 waits for those events, writes the summed milliseconds and the
 * launch counts per kind (0-2 FP64 Poisson, Hamiltonian, CMC; 3-5 their FP32
 * linearised forms) to ms_sum[6] / count[6] (host arrays) and restores graph
 * replay.  Errors: GR_ESTATE if unbound, GR_EINVAL for null outputs. */
int gr_sweep_timing(gr_grid g, int enable, double *ms_sum, int *count);

/* Low level, for step-by-step comparisons: `nsweeps` red-black Newton sweeps
 * of the finest level (even colour first) on field slot `field` with source
 * GR_RHS, coefficient GR_COEF and frozen scalars Fbar (Hamiltonian
 * regulariser <F>) and fshift (subtracted from the source). */
int gr_debug_sweep(gr_grid g, int kind, int field, double Fbar, double fshift, int nsweeps);

/* Low level: fine residual L(phi) - (f - fshift) of field slot `field` into
 * d_out (n^3 float64). */
int gr_debug_residual(gr_grid g, int kind, int field, double Fbar, double fshift, double *d_out);

/* ---- batched solve of many independent boxes ----
 * Many periodic boxes of uneven size (each an n^3 unit box, n even) solved
 * together: every phase of the cycle runs as one launch over all boxes, each
 * box stops on its own residual test (the single-grid criterion), and each
 * cycle's launch sequence is captured once per field in a hipGraph (only on a
 * non-null stream; GRMG_BATCH_GRAPH=0 disables it) and replayed.  Precision
 * GR_FP64, or GR_MIXED: the periodic boxes then run the single grid's
 * iterative refinement (FP64 residual and update, FP32 correction cycles whose
 * levels from 8^3 down run in FP64) without its FP64 fallback; patches stay
 * FP64.
 * Same memory rules as a single grid: the caller allocates
 * gr_batch_workspace_bytes() of device memory. */
typedef struct gr_batch_s *gr_batch;

/* Create a batch of `count` (1..4096) boxes described by descs[count], all
 * with the same code-unit parameters.  Host memory only. */
int gr_create_batch(const gr_grid_desc *descs, int count, const gr_params *prm, gr_batch *out);

/* A Dirichlet refinement patch (the refined levels of sec. 3, whose boundary
 * values come from the coarser level): n^3 cells (3 <= n <= 512) of spacing
 * h (0 < h <= 1e3) whose lower corner sits at origin[x,y,z] (box units,
 * |origin| <= 1e6) in the frame of its parent: the periodic box `parent`
 * (0 <= parent < nbox), or for nested refinement an earlier patch (parent =
 * nbox + j', j' below this patch's index), whose frame starts at that patch's
 * lower corner.  A nested patch must keep every interpolation sample strictly
 * between its parent's cell centres: per axis origin > (H + h)/2 and
 * origin + (n + 1/2) h < (N - 1/2) H for a parent of N cells of spacing H.
 * Anything else: GR_EINVAL.
 * Readings: levels halve while n is even and n/2 >= 3 (24..80 in steps of 8
 * end at 3, 4, 5, 3, 7, 4, 9, 5 cells); on every level the boundary value of
 * each boundary face is the parent's solved field at the face centre by
 * cell-centred trilinear interpolation (periodic in the parent), and the
 * 7-point stencil of a boundary cell takes 2b - phi_cell across that face;
 * the equations are the plain discrete ones (no regularisation terms, no
 * mean removed from the momentum sources, no zero-mean pin: those exist for
 * the periodic boundary, sec. 4.3.1-4.3.2); the coarsest level gets 32
 * red-black sweeps with no mean projection; the prolonged correction is odd
 * across every face.  Difference stencils of the source builders that reach
 * outside the patch read the parent's fields (and its A_ij) at those cells'
 * centres. */
typedef struct {
    int n;
    double h;
    int parent;
    double origin[3];
} gr_patch_desc;

/* A batch of nbox periodic boxes (items 0..nbox-1) and npatch patches (items
 * nbox..nbox+npatch-1), nbox + npatch <= 4096.  gr_batch_solve solves each
 * field of the patches right after that field of the boxes, nested patches
 * depth by depth (each depth from the finished field of the one above).
 * Every potential keeps its own array per item, so the coarser levels' fields
 * stay available after a solve.  set/get_field on a patch item move dense n^3
 * arrays (solved fields are stored padded internally). */
int gr_create_batch_patches(const gr_grid_desc *boxes, int nbox, const gr_patch_desc *patches, int npatch,
                            const gr_params *prm, gr_batch *out);
int gr_batch_workspace_bytes(gr_batch b, size_t *bytes);
/* Bind caller-owned device memory and a hipStream_t; zero-fills everything. */
int gr_batch_bind(gr_batch b, void *d_workspace, size_t bytes, void *hip_stream);
/* Copy one box's field (ids 0..15 as for a grid) from / to device memory. */
int gr_batch_set_field(gr_batch b, int item, int field, const void *d_src, int dtype);
int gr_batch_get_field(gr_batch b, int item, int field, void *d_dst, int dtype);
/* Solve the ten equations of every box from its sources (same order and
 * equations as gr_solve_constraints).  Optional host outputs:
 * cycles[count*10], rel_res[count*10] and item_seconds[count] (device-clock
 * time from the start of each field's solve until the box met its tolerance,
 * summed over the fields).  Returns the first non-OK box status. */
int gr_batch_solve(gr_batch b, const gr_solve_opts *opts, int *cycles, double *rel_res, double *item_seconds);
/* A sub-step of the refined levels (the parent code's adaptive time steps,
 * sec. 7): the ten equations of the patches only, from their current sources
 * (gr_batch_set_field on the patch items), with boundary and outside-stencil
 * values from the kept fields of the boxes and of the patches above them; the
 * boxes are neither read for their sources nor changed.  Outputs as
 * gr_batch_solve (a box's entries stay those of the last solve that ran it).
 * GR_EINVAL if the batch has no patches. */
int gr_batch_solve_patches(gr_batch b, const gr_solve_opts *opts, int *cycles, double *rel_res, double *item_seconds);
/* Tunes how each level of the periodic boxes is smoothed: for every depth
 * handled by grouped launches and every box side there with n >= 32 and
 * n % 16 == 0 it times one launch per colour, fused 16x16 tiles, and, where
 * the side allows, fused 32x16 tiles (n >= 64, n % 32 == 0) and fused 64x16
 * tiles (n >= 64, n % 64 == 0) on that side's boxes, and keeps the fastest.
 * All forms compute the same bits.  Uses field b of the boxes as scratch and
 * restores it; drops every captured cycle graph (FP64, mixed precision and
 * patches).  Writes one line per (depth,
 * side) to `report` (may be NULL).  Errors: GR_ESTATE if unbound. */
int gr_batch_autotune(gr_batch b, char *report, size_t report_bytes);
/* Per item and field of the last gr_batch_solve (h_flags, host, [items][10]):
 * 1 where mixed precision's refinement stalled (two steps in a row keeping
 * more than half of the FP64 residual, the single grid's rule; ratio from
 * GRMG_MIXED_STALL at creation) and the item finished that field with FP64
 * FAS cycles from its current iterate, 0 elsewhere (always 0 for FP64 solves
 * and for patches). */
int gr_batch_mixed_fallbacks(gr_batch b, int *h_flags);
/* Low level, for checks of the boundary values: writes the boundary values of
 * every level of every patch from their parents' current `field`, then copies
 * level `level` of patch `item`'s iterate, padded ((n_l+2)^3, x fastest; the
 * cells across the faces hold the boundary values) to d_dst. */
int gr_batch_debug_boundary(gr_batch b, int item, int field, int level, double *d_dst);
int gr_destroy_batch(gr_batch b);
const char *gr_batch_last_error(void);

/* ---- learned initial guess: a small 3-D U-Net ----
 * Levels with c[0..3] channels (c[0] = 16; c[1..3] in 16..64, multiples of
 * 16): two 3^3 convolutions + ReLU per level, 2x2x2 average pooling down,
 * nearest upsampling up with skip concatenation, and a 1x1 head.  Periodic
 * boundaries.  Convolutions run on BF16 matrix cores with FP32 accumulation;
 * parameters, gradients and Adam moments are FP32.  Inputs/outputs are planar
 * FP32 [channel][n^3] device arrays (x fastest), n a multiple of 32 up to
 * max_n.  Parameter vector order: per convolution (e0a, e0b, e1a, e1b, e2a,
 * e2b, e3a, e3b, d2a, d2b, d1a, d1b, d0a, d0b) weights [cout][27][cin]
 * (taps (dz,dy,dx) in {-1,0,1}^3, dx fastest) then bias [cout]; then the head
 * [out_ch][c0] and its bias. */
typedef struct gr_unet_s *gr_unet;
typedef struct {
    int in_ch, out_ch;
    int c[4];
    float lap_weight; /* loss = mean (y-t)^2 + lap_weight * mean (Lap(y-t))^2 (7-point,
                         periodic, unit spacing, per channel); 0: plain MSE */
    float clip_norm;  /* training: the gradient is scaled to at most this L2 norm before
                         each Adam step (a non-finite norm skips the step); 0: no clipping */
} gr_unet_desc;

int gr_unet_create(const gr_unet_desc *desc, int max_n, gr_unet *out);
int gr_unet_workspace_bytes(gr_unet u, size_t *bytes);
int gr_unet_param_count(gr_unet u, int64_t *count);
int gr_unet_bind(gr_unet u, void *d_workspace, size_t bytes, void *hip_stream);
/* He-normal weights from a counter-based generator (splitmix64 of seed and index). */
int gr_unet_init(gr_unet u, uint64_t seed);
int gr_unet_set_params(gr_unet u, const float *d_src);
int gr_unet_get_params(gr_unet u, float *d_dst);
/* d_out[out_ch][n^3] = network(d_in[in_ch][n^3]) */
int gr_unet_forward(gr_unet u, int n, const float *d_in, float *d_out);
/* Mean-square loss against d_target and its parameter gradient (copied to
 * d_grad[param_count] when not NULL); *h_loss (host) receives the loss. */
int gr_unet_loss_grad(gr_unet u, int n, const float *d_in, const float *d_target, float *d_grad, double *h_loss);
/* One Adam step (beta 0.9/0.999, eps 1e-8) with learning rate lr, on the
 * gradient clipped to the descriptor's clip_norm. */
int gr_unet_train_step(gr_unet u, int n, const float *d_in, const float *d_target, float lr, double *h_loss);
int gr_destroy_unet(gr_unet u);
const char *gr_unet_last_error(void);

/* ---- vector-mode extraction (sec. 6.2, the shift-vector power spectrum) ----
 * The shift beta^i (also B^i, and the momentum density s_i that sources it)
 * carries a scalar and a vector mode; a discrete curl removes the scalar
 * mode and k^2 P_V(k) = P_curl(k) gives the vector mode's power.
 * gr_vector_spectra takes three real FP64 fields v_x, v_y, v_z on the
 * periodic unit box (device arrays [z][y][x], x fastest, n^3 each, e.g. from
 * gr_get_field of GR_BETAX.., GR_BX.. or GR_SX..), forms the curl and the
 * divergence by 3-point central differences, transforms them with a 3-D FFT
 * on the device (F[g](m) = sum_x g(x) exp(-2 pi i m.x), integer m, k = 2 pi m)
 * and bins the modes in shells: shell j (0 <= j < nbins) holds the modes with
 * j + 1/2 <= |m| < j + 3/2.  Per mode P_curl = sum_i |F[(curl v)_i]|^2 / N^2,
 * P_div = |F[div v]|^2 / N^2 (N = n^3, box volume 1), and the vector- and
 * scalar-mode power of v itself P_vector = P_curl / |k_eff|^2, P_scalar =
 * P_div / |k_eff|^2 with k_eff,i = n sin(2 pi m_i / n), the central
 * difference's symbol (so P_vector + P_scalar is v's own power per mode).
 * h_out (host, [6][nbins]) receives per shell the mean |k|, the mode count,
 * and the means of P_curl, P_div, P_vector, P_scalar over its modes.  nbins =
 * n / 8 reaches a quarter of the Nyquist wave number pi n.
 * Handle: n a power of two in [8, 1024], 1 <= nbins <= n / 4; the workspace
 * (two complex n^3 arrays plus small tables, gr_spectra_workspace_bytes,
 * 256-byte aligned) is the caller's.  gr_vector_spectra runs on the bound
 * stream and synchronises it before returning; the results are deterministic
 * (fixed summation order).  gr_spectra_fft: in-place forward 3-D FFT of an
 * n^3 complex array (interleaved re, im doubles) with the same kernels.
 * Errors: GR_EINVAL (null, sizes, alignment), GR_ESTATE (unbound), GR_EDEVICE. */
typedef struct gr_spectra_s *gr_spectra;
int gr_create_spectra(int n, int nbins, gr_spectra *out);
int gr_spectra_workspace_bytes(gr_spectra s, size_t *bytes);
int gr_spectra_bind(gr_spectra s, void *d_workspace, size_t bytes, void *hip_stream);
int gr_vector_spectra(gr_spectra s, const double *d_vx, const double *d_vy, const double *d_vz, double *h_out);
int gr_spectra_fft(gr_spectra s, double *d_data);
int gr_destroy_spectra(gr_spectra s);
const char *gr_spectra_last_error(void);

/* Destroy a handle (the workspace stays the caller's). NULL is accepted. */
int gr_destroy_grid(gr_grid g);

/* Thread-local message of the last failing call on this thread. */
const char *gr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GR_H */
