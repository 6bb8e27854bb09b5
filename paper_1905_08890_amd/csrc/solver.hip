// C ABI (include/gr.h) and host orchestration of the multigrid solve:
// workspace layout, the FAS V-cycle schedule, cycle control with the
// stopping test, and the ten-field dependency order of the paper's
// solution scheme (sec. 2.4; equations of sec. 4.3).
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <functional>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "gr_internal.h"

using namespace grmg;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(GR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

#define LAUNCHCHK()                                                                               \
    do {                                                                                          \
        hipError_t e_ = hipGetLastError();                                                        \
        if (e_ != hipSuccess) return fail(GR_EDEVICE, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                                                                                 \
    do {                                                                                          \
        int st_ = (expr);                                                                         \
        if (st_ != GR_OK) return st_;                                                             \
    } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

} // namespace

struct gr_grid_s {
    int n = 0;
    double h = 0.0;
    gr_params prm{};
    int nlev = 0;
    Level lev[kMaxLevels]{};
    Level32 lev32[kMaxLevels]{}; // FP32 correction-cycle arrays (mixed precision)
    // fine-level arrays
    double *field[10]{};
    double *src[5]{}; // s0, sx, sy, sz, sm
    double *A6[6]{};
    double *AA = nullptr;
    double *fB[3]{}; // sources of B^i (kept for the three solves)
    double *alt[10]{}; // alternative (previous-step) guesses, saved by gr_set_guess
    bool alt_valid[10]{};
    double *hist[10]{}; // history: each field as it was before the last GR_SET_EXTRAP guess
    bool hist_valid[10]{};
    double *gtmp = nullptr; // 3/4 of a fine array: cubic guess interpolation passes
    // Helper hierarchies (levels, FP32 levels, reductions, stream) that solve
    // components 1 and 2 of a vector equation concurrently with component 0.
    bool solver_only = false;
    gr_grid_s *sub[2]{};
    void *cic = nullptr;    // cell-ordered deposit scratch for up to n^3 particles
    double *partials = nullptr;
    double *scal = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool fused = true;     // fused tile smoother on large levels
    FusedCfg fcfg;
    FusedCfg tuned[kMaxLevels][6]; // per level and kind (0-2 FP64, 3-5 FP32), set by gr_autotune
    bool tuned_ok[kMaxLevels][6]{};
    bool tuned_split[kMaxLevels][6]{}; // the tuner found one launch per colour faster
    int coarse_n = 8;      // levels with n <= coarse_n run in one single-workgroup launch
    int coarse_n32 = 8;    // the same for the FP32 correction cycles
    int coarse_np = 16;    // the same threshold for the Poisson kind (FP64 and correction cycles): its point
                           // update is cheap enough for one CU to take a 16^3 level faster than ~11 launches
    int skew = 0;          // workspace array skew in bytes (see layout)
    double stall_ratio = 0.5; // mixed precision: a refinement step that keeps more than this
                              // fraction of the residual counts as stalled (two in a row: FP64)
    size_t ws_bytes = 0;
    // Solves run on a private stream (joined to the caller's by events) so that
    // each cycle body can be captured once into a hipGraph and replayed.
    hipStream_t user_stream = nullptr;
    hipStream_t work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // per-cycle read-back of the two stopping norms: page-locked coherent host
    // slots that the norm finalize writes directly (d_norms: their device
    // address), and an event the host spins on (set up at bind; absent on the
    // static grid)
    double *h_norms = nullptr, *d_norms = nullptr;
    hipEvent_t ev_norms = nullptr;
    bool use_graph = true;
    struct GraphEntry {
        int prec, kind, nu1, nu2;
        const double *phi;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    // optional timing of finest-level fused sweeps (gr_sweep_timing)
    bool timing = false, graph_saved = true;
    struct SweepEv {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<SweepEv> sweep_ev;
    std::vector<hipEvent_t> ev_free;

    void drop_graphs()
    {
        for (auto &e : graphs) (void)hipGraphExecDestroy(e.exec);
        graphs.clear();
    }
    ~gr_grid_s()
    {
        for (auto *h : sub) delete h;
        drop_graphs();
        for (auto &e : sweep_ev) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
        for (auto e : ev_free) (void)hipEventDestroy(e);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (ev_norms) (void)hipEventDestroy(ev_norms);
        if (h_norms) (void)hipHostFree(h_norms);
        if (work) (void)hipStreamDestroy(work);
    }

    long N() const { return (long)n * n * n; }
    OpConst oc() const
    {
        OpConst o;
        o.kappa = 1.0 / (2.0 * prm.a * prm.a * prm.c_tilde * prm.c_tilde);
        o.A = 1.5 * prm.a * prm.omega_m;
        return o;
    }
};

namespace {

int num_levels(int n)
{
    int L = 1;
    while (n % 4 == 0) {
        n /= 2;
        ++L;
    }
    return L;
}

// Carve the workspace; with base == nullptr only count bytes.
size_t layout(gr_grid g, char *base)
{
    size_t off = 0;
    int count = 0;
    // Arrays of one size would otherwise start at identical address bits modulo
    // their (power-of-two) length; a rotating skew of `skew` bytes per array
    // keeps the streams of one kernel from hitting the same HBM channels in step.
    auto take = [&](size_t bytes) -> double * {
        double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
        off += align_up(bytes) + align_up((size_t)g->skew * (size_t)(count++ % 8));
        return p;
    };
    const size_t fb = sizeof(double) * (size_t)g->N();
    if (!g->solver_only) {
        for (int f = 0; f < 10; ++f) g->field[f] = take(fb);
        for (int s = 0; s < 5; ++s) g->src[s] = take(fb);
        for (int c = 0; c < 6; ++c) g->A6[c] = take(fb);
        g->AA = take(fb);
        for (int c = 0; c < 3; ++c) g->fB[c] = take(fb);
        for (int f = 0; f < 10; ++f) g->alt[f] = take(fb);
        for (int f = 0; f < 10; ++f) g->hist[f] = take(fb);
        g->gtmp = take(3 * fb / 4);
        g->cic = take(cic_sorted_bytes(g->N(), g->N()));
    }
    for (int l = 0; l < g->nlev; ++l) {
        Level &L = g->lev[l];
        const size_t lb = sizeof(double) * (size_t)L.N;
        L.phi = (l == 0) ? nullptr : take(lb);
        L.phi0 = take(lb);
        L.f = take(lb);
        L.coef = take(lb);
        L.tmp = take(lb);
    }
    for (int l = 0; l < g->nlev; ++l) {
        Level32 &V = g->lev32[l];
        const size_t lb = sizeof(float) * (size_t)g->lev[l].N;
        V.e = reinterpret_cast<float *>(take(lb));
        V.b = reinterpret_cast<float *>(take(lb));
        V.a = reinterpret_cast<float *>(take(lb));
        V.c = reinterpret_cast<float *>(take(lb));
        V.tmp = reinterpret_cast<float *>(take(lb));
    }
    g->partials = take(sizeof(double) * kReduceBlocks * 4);
    g->scal = take(sizeof(double) * S_NUM);
    for (auto *h : g->sub)
        if (h) off += align_up(layout(h, base ? base + off : nullptr));
    return off;
}

// ------------------------------------------------------------ reductions

int reduce_mean(gr_grid g, const double *x, const double *y, long N, double *out)
{
    launch_sum(g->stream, x, y, N, g->partials);
    launch_finalize(g->stream, g->partials, 1, 1.0 / (double)N, nullptr, out);
    LAUNCHCHK();
    return GR_OK;
}

// pin: phi -= mean(phi)
int pin_mean(gr_grid g, double *phi, long N)
{
    CHK(reduce_mean(g, phi, nullptr, N, g->scal + S_MEAN));
    launch_sub_scalar(g->stream, phi, N, g->scal + S_MEAN);
    LAUNCHCHK();
    return GR_OK;
}

// Reads the sums of eps^2 and f^2 of the stopping test (slots S_RN, S_FN) to
// the host once the work queued before it is done.  On a bound grid the
// finalize that produced them (always the last kernel before this call) also
// wrote them to the page-locked coherent slots h_norms, and the host spins on an
// event (no copy, no sleeping wait between V-cycles); otherwise it copies and
// waits on the stream.
int read_norms(gr_grid g, double out[2])
{
    if (g->d_norms && g->ev_norms) { // the norm finalize wrote them to h_norms
        HIPCHK(hipEventRecord(g->ev_norms, g->stream));
        hipError_t e;
        while ((e = hipEventQuery(g->ev_norms)) == hipErrorNotReady) {
        }
        if (e != hipSuccess) return fail(GR_EDEVICE, "norm read-back: %s", hipGetErrorString(e));
        const volatile double *h = g->h_norms;
        out[0] = h[0];
        out[1] = h[1];
        return GR_OK;
    }
    HIPCHK(hipMemcpyAsync(out, g->scal + S_RN, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    HIPCHK(hipStreamSynchronize(g->stream));
    return GR_OK;
}

// ------------------------------------------------------ graphs and streams

// Run `body` (kernel launches only, no host synchronisation) on the work
// stream: captured into a hipGraph on first use for this key, replayed after.
template <class F>
int run_captured(gr_grid g, int prec, int kind, int nu1, int nu2, const double *phi, F body)
{
    if (!g->use_graph) return body();
    hipGraphExec_t exec = nullptr;
    for (auto &e : g->graphs)
        if (e.prec == prec && e.kind == kind && e.nu1 == nu1 && e.nu2 == nu2 && e.phi == phi) exec = e.exec;
    if (!exec) {
        hipGraph_t gr;
        HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
        const int st = body();
        hipError_t e = hipStreamEndCapture(g->stream, &gr);
        if (st != GR_OK) {
            if (e == hipSuccess) (void)hipGraphDestroy(gr);
            return st;
        }
        if (e != hipSuccess) return fail(GR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(GR_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        g->graphs.push_back({prec, kind, nu1, nu2, phi, exec});
    }
    HIPCHK(hipGraphLaunch(exec, g->stream));
    return GR_OK;
}

// Moves a solve onto the work stream: it starts after the work already queued
// on the caller's stream, and the caller's stream waits for it at the end.
struct WorkScope {
    gr_grid g;
    bool ok = false;
    explicit WorkScope(gr_grid g_) : g(g_)
    {
        if (hipEventRecord(g->ev_in, g->user_stream) != hipSuccess) return;
        if (hipStreamWaitEvent(g->work, g->ev_in, 0) != hipSuccess) return;
        g->stream = g->work;
        ok = true;
    }
    ~WorkScope()
    {
        if (!ok) return;
        (void)hipEventRecord(g->ev_out, g->work);
        (void)hipStreamWaitEvent(g->user_stream, g->ev_out, 0);
        g->stream = g->user_stream;
    }
};

// ------------------------------------------------------------ V-cycle

struct EqCtx {
    int kind;
    OpConst oc;
    int nu1, nu2;
};

const double *fbar_ptr(gr_grid g, int l) { return g->scal + (l == 0 ? S_FBAR : S_ZERO); }
const double *fshift_ptr(gr_grid g, int l) { return g->scal + (l == 0 ? S_FSHIFT : S_ZERO); }

// launch configuration of the fused sweep on level l for a kind (0..5)
const FusedCfg &fused_cfg(gr_grid g, int l, int kind)
{
    return g->tuned_ok[l][kind] ? g->tuned[l][kind] : g->fcfg;
}

// fused or one launch per colour on level l: the tuner's choice, else by size
bool use_fused(gr_grid g, int l, int kind)
{
    if (!g->fused) return false;
    if (g->tuned_ok[l][kind]) return !g->tuned_split[l][kind];
    return fused_sweep_ok(g->lev[l].n, g->fcfg.min_n);
}

hipEvent_t pooled_event(gr_grid g)
{
    if (!g->ev_free.empty()) {
        hipEvent_t e = g->ev_free.back();
        g->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one finest-level fused sweep launch, bracketed by events when timing.
template <class F>
void timed_sweep(gr_grid g, int l, int kind, F launch)
{
    if (!g->timing || l != 0) {
        launch();
        return;
    }
    hipEvent_t a = pooled_event(g), b = pooled_event(g);
    if (!a || !b) {
        launch();
        return;
    }
    (void)hipEventRecord(a, g->stream);
    launch();
    (void)hipEventRecord(b, g->stream);
    g->sweep_ev.push_back({kind, a, b});
}

// nsweeps red-black sweeps of level l on L.phi.  The fused kernels work out
// of place, alternating between L.phi and L.tmp; after an odd number of
// launches the two pointers are exchanged, so the iterate is L.phi again (the
// V-cycle of the level puts them back, copying only if its launches were odd).
int smooth(gr_grid g, const EqCtx &E, int l, int nsweeps)
{
    Level &L = g->lev[l];
    hipStream_t s = g->stream;
    if (nsweeps <= 0) return GR_OK;
    if (!use_fused(g, l, E.kind)) {
        for (int it = 0; it < nsweeps; ++it)
            launch_rb_sweep(E.kind, s, L.phi, L.f, L.coef, L.n, L.h, E.oc, fbar_ptr(g, l), fshift_ptr(g, l));
        LAUNCHCHK();
        return GR_OK;
    }
    double *a = L.phi, *b = L.tmp;
    const FusedCfg &cfg = fused_cfg(g, l, E.kind);
    for (int it = 0; it < nsweeps; ++it) {
        timed_sweep(g, l, E.kind, [&] {
            launch_rb_fused(E.kind, s, a, b, L.f, L.coef, L.n, L.h, E.oc, fbar_ptr(g, l), fshift_ptr(g, l), cfg);
        });
        double *t = a;
        a = b;
        b = t;
    }
    if (a != L.phi) std::swap(L.phi, L.tmp);
    LAUNCHCHK();
    return GR_OK;
}

int vcycle_body(gr_grid g, const EqCtx &E, int l);

// Every V-cycle leaves the iterate of its level in the array it found it in.
int vcycle(gr_grid g, const EqCtx &E, int l)
{
    Level &L = g->lev[l];
    double *orig = L.phi;
    const int st = vcycle_body(g, E, l);
    if (L.phi != orig) {
        launch_copy(g->stream, orig, L.phi, L.N);
        L.tmp = L.phi;
        L.phi = orig;
        LAUNCHCHK();
    }
    return st;
}

int vcycle_body(gr_grid g, const EqCtx &E, int l)
{
    Level &L = g->lev[l];
    hipStream_t s = g->stream;
    if (L.n <= (E.kind == GR_KIND_POISSON ? g->coarse_np : g->coarse_n)) {
        CoarseLevelsT<double> C;
        C.nl = g->nlev - l;
        for (int i = 0; i < C.nl; ++i) {
            const Level &V = g->lev[l + i];
            C.n[i] = V.n;
            C.inv_h2[i] = 1.0 / (V.h * V.h);
            C.phi[i] = V.phi;
            C.phi0[i] = V.phi0;
            C.f[i] = V.f;
            C.c1[i] = V.coef;
            C.c2[i] = nullptr;
            C.tmp[i] = V.tmp;
        }
        launch_coarse_vcycle(E.kind, s, C, E.nu1, E.nu2, E.oc, fbar_ptr(g, l), fshift_ptr(g, l));
        LAUNCHCHK();
        return GR_OK;
    }
    if (l == g->nlev - 1) {
        // coarsest: 32 sweeps, then remove the mean of the correction
        launch_copy(s, L.tmp, L.phi, L.N);
        for (int it = 0; it < kCoarseSweeps; ++it)
            launch_rb_sweep(E.kind, s, L.phi, L.f, L.coef, L.n, L.h, E.oc, fbar_ptr(g, l), fshift_ptr(g, l));
        CHK(reduce_mean(g, L.phi, L.tmp, L.N, g->scal + S_MEAN));
        launch_sub_scalar(s, L.phi, L.N, g->scal + S_MEAN);
        LAUNCHCHK();
        return GR_OK;
    }
    CHK(smooth(g, E, l, E.nu1));
    Level &C = g->lev[l + 1];
    // R phi -> C.phi and C.phi0; R eps -> C.tmp; then f^H = L^H(R phi) - R eps
    launch_residual_restrict(E.kind, s, L.phi, L.f, L.coef, L.n, L.h, E.oc, fbar_ptr(g, l), fshift_ptr(g, l),
                             C.phi, C.phi0, C.tmp);
    launch_coarse_rhs(E.kind, s, C.phi, C.coef, C.tmp, C.n, C.h, E.oc, C.f);
    LAUNCHCHK();
    CHK(vcycle(g, E, l + 1));
    // phi += P e with the coarse correction e = phi^H - R phi formed on the fly
    launch_prolong_correct(s, L.phi, L.n, C.phi, C.phi0);
    LAUNCHCHK();
    return smooth(g, E, l, E.nu2);
}

// Solve one equation for `phi` (fine), with fine source lev[0].f and fine
// coefficient lev[0].coef already in place.  Follows the cycle definition:
// pin the guess; per cycle: frozen means, residual norm, stopping test,
// V-cycle, pin.
int solve_one(gr_grid g, int kind, double *phi, const gr_solve_opts &o, int *cycles_out, double *rel_out)
{
    const long N = g->N();
    Level &F = g->lev[0];
    F.phi = phi;
    EqCtx E{kind, g->oc(), o.nu1, o.nu2};
    if (kind != GR_KIND_POISSON)
        for (int l = 1; l < g->nlev; ++l)
            launch_restrict(g->stream, g->lev[l - 1].coef, g->lev[l - 1].n, g->lev[l].coef);
    launch_set_scalar(g->stream, g->scal + S_FBAR, 0.0);
    launch_set_scalar(g->stream, g->scal + S_FSHIFT, 0.0);
    if (kind == GR_KIND_CMC) CHK(reduce_mean(g, F.f, nullptr, N, g->scal + S_FMEAN));
    LAUNCHCHK();
    CHK(pin_mean(g, phi, N));

    // frozen means of this iterate, then the two norms of the stopping test
    auto measure = [&]() -> int {
        hipStream_t s = g->stream;
        if (kind == GR_KIND_HAMILTONIAN) {
            launch_sum_ham_F(s, phi, F.f, F.coef, N, E.oc, g->partials);
            launch_finalize(s, g->partials, 1, 1.0 / (double)N, nullptr, g->scal + S_FBAR);
        } else if (kind == GR_KIND_CMC) {
            launch_sum_prod(s, F.coef, phi, N, g->partials);
            launch_finalize(s, g->partials, 1, 1.0 / (double)N, g->scal + S_FMEAN, g->scal + S_FSHIFT);
        }
        launch_res_norms(kind, s, phi, F.f, F.coef, F.n, F.h, E.oc, g->scal + S_FBAR, g->scal + S_FSHIFT,
                         g->partials);
        launch_finalize(s, g->partials, 2, 1.0 / (double)N, nullptr, g->scal + S_RN, g->d_norms);
        LAUNCHCHK();
        return GR_OK;
    };
    // one V-cycle (pinned for the nonlinear kinds), then the next measurement
    auto cycle = [&]() -> int {
        CHK(vcycle(g, E, 0));
        // The Poisson V-cycle commutes with adding a constant (the Laplacian, the
        // smoother, R and P all do, and the coarsest level removes the mean of
        // its correction), and so does the stopping quantity: pinning once at the
        // end gives the per-cycle pinned iterate up to rounding.
        if (kind != GR_KIND_POISSON) CHK(pin_mean(g, phi, N));
        return measure();
    };

    CHK(measure());
    int cyc = 0;
    double rel = 0.0;
    int st = GR_OK;
    for (;;) {
        double hn[2];
        CHK(read_norms(g, hn));
        const double rn = std::sqrt(hn[0]), fn = std::sqrt(hn[1]);
        rel = rn / (fn > 0.0 ? fn : 1.0);
        if (!std::isfinite(rel)) {
            st = fail(GR_ENAN, "non-finite residual (kind %d, cycle %d)", kind, cyc);
            break;
        }
        if (o.rtol > 0.0 && (rel <= o.rtol || rn == 0.0)) break;
        if (cyc >= o.max_cycles) {
            if (o.rtol > 0.0)
                st = fail(GR_ENOTCONV, "kind %d: rel residual %.3e after %d cycles", kind, rel, cyc);
            break;
        }
        CHK(run_captured(g, GR_FP64, kind, o.nu1, o.nu2, phi, cycle));
        ++cyc;
    }
    if (kind == GR_KIND_POISSON && cyc > 0) CHK(pin_mean(g, phi, N));
    *cycles_out = cyc;
    *rel_out = rel;
    return st;
}

// ------------------------------------------------- mixed precision (FP32 inner)

// nsweeps sweeps of the linearised FP32 correction equation on level l.
// e_is_zero: the correction is identically zero on entry (not yet written).
int smooth32(gr_grid g, int lkind, int l, int nsweeps, OpConst oc, bool e_is_zero)
{
    Level &L = g->lev[l];
    Level32 &V = g->lev32[l];
    hipStream_t s = g->stream;
    const double *zero = g->scal + S_ZERO;
    if (!use_fused(g, l, lkind)) {
        if (e_is_zero) launch_fill_f32(s, V.e, L.N);
        for (int it = 0; it < nsweeps; ++it) launch_rb_sweep_f32(lkind, s, V.e, V.b, V.c, V.a, L.n, L.h, oc, zero);
        LAUNCHCHK();
        return GR_OK;
    }
    if (e_is_zero && nsweeps == 0) launch_fill_f32(s, V.e, L.N);
    float *a = V.e, *b = V.tmp;
    const FusedCfg &cfg = fused_cfg(g, l, lkind);
    for (int it = 0; it < nsweeps; ++it) {
        const float *in = (it == 0 && e_is_zero) ? nullptr : a;
        timed_sweep(g, l, lkind, [&] { launch_rb_fused_f32(lkind, s, in, b, V.b, V.c, V.a, L.n, L.h, oc, zero, cfg); });
        float *t = a;
        a = b;
        b = t;
    }
    if (a != V.e) std::swap(V.e, V.tmp); // put back by the level's V-cycle
    LAUNCHCHK();
    return GR_OK;
}

// Correction-scheme V-cycle for J e = b on levels l.. (e = 0 on entry at every
// level; on level l it may be unwritten when e_unset): sweeps, b^H = R(b - J e),
// recursion, e += P e^H, sweeps; the coarsest level (always inside the
// single-workgroup kernel) does 32 sweeps and removes the mean of its correction.
int vcycle32_body(gr_grid g, int lkind, int l, int nu1, int nu2, OpConst oc, bool e_unset);

// Every correction V-cycle leaves the correction of its level in the array it
// found it in.
int vcycle32(gr_grid g, int lkind, int l, int nu1, int nu2, OpConst oc, bool e_unset)
{
    Level32 &V = g->lev32[l];
    float *orig = V.e;
    const int st = vcycle32_body(g, lkind, l, nu1, nu2, oc, e_unset);
    if (V.e != orig) {
        launch_copy_f32(g->stream, orig, V.e, g->lev[l].N);
        V.tmp = V.e;
        V.e = orig;
        LAUNCHCHK();
    }
    return st;
}

int vcycle32_body(gr_grid g, int lkind, int l, int nu1, int nu2, OpConst oc, bool e_unset)
{
    Level &L = g->lev[l];
    Level32 &V = g->lev32[l];
    hipStream_t s = g->stream;
    if (L.n <= (lkind == K_LIN_POISSON ? g->coarse_np : g->coarse_n32) || l == g->nlev - 1) {
        if (e_unset) launch_fill_f32(s, V.e, L.N);
        CoarseLevelsT<float> C;
        C.nl = g->nlev - l;
        for (int i = 0; i < C.nl; ++i) {
            const Level &Q = g->lev[l + i];
            const Level32 &W = g->lev32[l + i];
            C.n[i] = Q.n;
            C.inv_h2[i] = 1.0 / (Q.h * Q.h);
            C.phi[i] = W.e;
            C.phi0[i] = nullptr;
            C.f[i] = W.b;
            C.c1[i] = W.c;
            C.c2[i] = W.a;
            C.tmp[i] = W.tmp;
        }
        launch_coarse_vcycle_f32(lkind, s, C, nu1, nu2, oc, g->scal + S_ZERO);
        LAUNCHCHK();
        return GR_OK;
    }
    CHK(smooth32(g, lkind, l, nu1, oc, e_unset));
    Level32 &C = g->lev32[l + 1];
    launch_lin_residual_restrict_f32(lkind, s, V.e, V.b, V.c, V.a, L.n, L.h, oc, C.b, C.e);
    LAUNCHCHK();
    CHK(vcycle32(g, lkind, l + 1, nu1, nu2, oc, false));
    launch_prolong_add_f32(s, V.e, L.n, C.e);
    LAUNCHCHK();
    return smooth32(g, lkind, l, nu2, oc, false);
}

// Mixed-precision iterative refinement for one equation: each outer step
// evaluates the FP64 residual (and stopping test) of the regularised fine
// equation exactly as the FP64 cycle does, solves the linearised correction
// J(phi) e = -r approximately by one FP32 V-cycle from e = 0, and updates
// phi <- phi + e - <e> in FP64 (the zero-mean pin folded into the update).
// If the FP64 residual stops falling (ratio above stall_ratio, 0.5 by default,
// twice in a row) the field continues with FP64 FAS cycles.
int solve_one_mixed(gr_grid g, int kind, double *phi, const gr_solve_opts &o, int *cycles_out, double *rel_out,
                    int *fell_back)
{
    hipStream_t s = g->stream;
    const long N = g->N();
    Level &F = g->lev[0];
    Level32 &F32 = g->lev32[0];
    F.phi = phi;
    const OpConst oc = g->oc();
    const int lkind = kind + K_LIN_POISSON;
    *fell_back = 0;
    launch_set_scalar(s, g->scal + S_FBAR, 0.0);
    launch_set_scalar(s, g->scal + S_FSHIFT, 0.0);
    if (kind == GR_KIND_CMC) {
        CHK(reduce_mean(g, F.f, nullptr, N, g->scal + S_FMEAN));
        launch_neg_to_f32(s, F32.c, F.coef, N);
        for (int l = 1; l < g->nlev; ++l) launch_restrict_f32(s, g->lev32[l - 1].c, g->lev[l - 1].n, g->lev32[l].c);
    }
    LAUNCHCHK();
    CHK(pin_mean(g, phi, N));

    // Poisson: the update phi + e and the next residual are one pass, out of
    // place, alternating between the field and the finest level's scratch
    // array (the iterate is copied back to the field at the end)
    const bool fuse_update = kind == GR_KIND_POISSON;
    double *cur = phi, *other = F.tmp;
    // frozen means (their sums already in the partials when `summed`), FP64
    // residual (as FP32 right-hand side) and the stopping norms
    auto measure = [&](bool summed = false) -> int {
        if (kind == GR_KIND_HAMILTONIAN) {
            if (!summed) launch_sum_ham_F(s, phi, F.f, F.coef, N, oc, g->partials);
            launch_finalize(s, g->partials, 1, 1.0 / (double)N, nullptr, g->scal + S_FBAR);
        } else if (kind == GR_KIND_CMC) {
            if (!summed) launch_sum_prod(s, F.coef, phi, N, g->partials);
            launch_finalize(s, g->partials, 1, 1.0 / (double)N, g->scal + S_FMEAN, g->scal + S_FSHIFT);
        }
        launch_ir_residual(kind, s, cur, F.f, F.coef, F.n, F.h, oc, g->scal + S_FBAR, g->scal + S_FSHIFT, F32.b, F32.a,
                           F32.c, g->partials);
        launch_finalize(s, g->partials, 2, 1.0 / (double)N, nullptr, g->scal + S_RN, g->d_norms);
        LAUNCHCHK();
        return GR_OK;
    };
    // one FP32 correction cycle and the FP64 update, then the next measurement
    auto step = [&]() -> int {
        if (kind == GR_KIND_HAMILTONIAN) { // a and c on every level: one launch per level above 32^3, then one
            int l = 1;
            for (; l < g->nlev && g->lev[l - 1].n > 32; ++l)
                launch_restrict2_f32(s, g->lev32[l - 1].a, g->lev32[l - 1].c, g->lev[l - 1].n, g->lev32[l].a,
                                     g->lev32[l].c);
            if (l < g->nlev) {
                RestrictChain R{};
                R.nl = g->nlev - l;
                for (int i = 0; i <= R.nl; ++i) {
                    R.n[i] = g->lev[l - 1 + i].n;
                    R.a[i] = g->lev32[l - 1 + i].a;
                    R.c[i] = g->lev32[l - 1 + i].c;
                }
                launch_restrict2_chain(s, R);
            }
        }
        CHK(vcycle32(g, lkind, 0, o.nu1, o.nu2, oc, true));
        if (fuse_update) { // shift-invariant: one pin at the end (as in the FP64 cycle)
            launch_ir_update_residual(s, cur, F32.e, other, F.f, F.n, F.h, oc, g->scal + S_FBAR, g->scal + S_FSHIFT,
                                      F32.b, g->partials);
            launch_finalize(s, g->partials, 2, 1.0 / (double)N, nullptr, g->scal + S_RN, g->d_norms);
            LAUNCHCHK();
            return GR_OK;
        } else { // the update fused with the next frozen-mean sum
            launch_sum_f32(s, F32.e, N, g->partials);
            launch_finalize(s, g->partials, 1, 1.0 / (double)N, nullptr, g->scal + S_MEAN);
            launch_ir_update_sum(kind, s, phi, F32.e, g->scal + S_MEAN, F.f, F.coef, N, oc, g->partials);
        }
        LAUNCHCHK();
        return measure(true);
    };

    CHK(measure());
    int cyc = 0, stall = 0;
    double rel = 0.0, prev = HUGE_VAL;
    int st = GR_OK;
    for (;;) {
        double hn[2];
        CHK(read_norms(g, hn));
        const double rn = std::sqrt(hn[0]), fn = std::sqrt(hn[1]);
        rel = rn / (fn > 0.0 ? fn : 1.0);
        if (!std::isfinite(rel)) {
            st = fail(GR_ENAN, "non-finite residual (kind %d, refinement step %d)", kind, cyc);
            break;
        }
        if (o.rtol > 0.0 && (rel <= o.rtol || rn == 0.0)) break;
        if (cyc >= o.max_cycles) {
            if (o.rtol > 0.0)
                st = fail(GR_ENOTCONV, "kind %d: rel residual %.3e after %d refinement steps", kind, rel, cyc);
            break;
        }
        stall = rel > g->stall_ratio * prev ? stall + 1 : 0;
        prev = rel;
        if (stall >= 2) { // FP32 corrections no longer help: finish in FP64
            *fell_back = 1;
            if (cur != phi) {
                launch_copy(s, phi, cur, N);
                LAUNCHCHK();
                cur = phi;
            }
            gr_solve_opts o2 = o;
            o2.max_cycles = o.max_cycles - cyc;
            int c2 = 0;
            st = solve_one(g, kind, phi, o2, &c2, &rel);
            cyc += c2;
            break;
        }
        // graphs keyed by the field and by which array holds the iterate
        CHK(run_captured(g, GR_MIXED, kind + (cur != phi ? 16 : 0), o.nu1, o.nu2, phi, step));
        if (fuse_update) std::swap(cur, other);
        ++cyc;
    }
    if (cur != phi) {
        launch_copy(s, phi, cur, N);
        LAUNCHCHK();
    }
    if (kind == GR_KIND_POISSON && cyc > 0 && !*fell_back) CHK(pin_mean(g, phi, N));
    *cycles_out = cyc;
    *rel_out = rel;
    return st;
}

int solve_field(gr_grid g, int kind, double *phi, const gr_solve_opts &o, int *cycles, double *rel, int *fell_back)
{
    *fell_back = 0;
    if (o.precision == GR_MIXED) return solve_one_mixed(g, kind, phi, o, cycles, rel, fell_back);
    return solve_one(g, kind, phi, o, cycles, rel);
}

// The stopping quantity rms(eps)/rms(f) of an iterate phi (pinned here), with
// the frozen means evaluated from it, exactly as at the start of a cycle.
// Uses the fine source and coefficient already in place.
int guess_residual(gr_grid g, int kind, double *phi, double *rel_out)
{
    hipStream_t s = g->stream;
    const long N = g->N();
    Level &F = g->lev[0];
    const OpConst oc = g->oc();
    CHK(pin_mean(g, phi, N));
    launch_set_scalar(s, g->scal + S_FBAR, 0.0);
    launch_set_scalar(s, g->scal + S_FSHIFT, 0.0);
    if (kind == GR_KIND_HAMILTONIAN) {
        launch_sum_ham_F(s, phi, F.f, F.coef, N, oc, g->partials);
        launch_finalize(s, g->partials, 1, 1.0 / (double)N, nullptr, g->scal + S_FBAR);
    } else if (kind == GR_KIND_CMC) {
        CHK(reduce_mean(g, F.f, nullptr, N, g->scal + S_FMEAN));
        launch_sum_prod(s, F.coef, phi, N, g->partials);
        launch_finalize(s, g->partials, 1, 1.0 / (double)N, g->scal + S_FMEAN, g->scal + S_FSHIFT);
    }
    launch_res_norms(kind, s, phi, F.f, F.coef, F.n, F.h, oc, g->scal + S_FBAR, g->scal + S_FSHIFT, g->partials);
    launch_finalize(s, g->partials, 2, 1.0 / (double)N, nullptr, g->scal + S_RN, g->d_norms);
    LAUNCHCHK();
    double hn[2];
    CHK(read_norms(g, hn));
    const double rn = std::sqrt(hn[0]), fn = std::sqrt(hn[1]);
    *rel_out = rn / (fn > 0.0 ? fn : 1.0);
    return GR_OK;
}

// GR_GUESS_CHECKED: keep the held guess unless the saved alternative (the
// previous-step field) has a smaller stopping quantity, or the held guess is
// not finite; returns 1 when the alternative was taken.
// on hierarchy h (whose fine source and coefficient are in place)
int choose_guess_on(gr_grid h, int kind, double *phi, double *alt, bool valid, int *took_alt, double *rel_held,
                    double *rel_alt)
{
    *took_alt = 0;
    if (!valid) return GR_OK;
    double r_held = 0.0, r_alt = 0.0;
    CHK(guess_residual(h, kind, phi, &r_held));
    CHK(guess_residual(h, kind, alt, &r_alt));
    *rel_held = r_held;
    *rel_alt = r_alt;
    if (!(r_held < r_alt)) {
        launch_copy(h->stream, phi, alt, h->N());
        LAUNCHCHK();
        *took_alt = 1;
    }
    return GR_OK;
}

int choose_guess(gr_grid g, int kind, int fid, int *took_alt, double *rel_held, double *rel_alt)
{
    return choose_guess_on(g, kind, g->field[fid], g->alt[fid], g->alt_valid[fid], took_alt, rel_held, rel_alt);
}

int check_opts(const gr_solve_opts *o)
{
    if (!o) return fail(GR_EINVAL, "null opts");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 64 || o->nu2 > 64 || o->max_cycles < 0 || o->max_cycles > 100000)
        return fail(GR_EINVAL, "bad cycle options");
    if (!(o->rtol == o->rtol)) return fail(GR_EINVAL, "rtol is NaN");
    if (o->precision != GR_FP64 && o->precision != GR_MIXED) return fail(GR_EINVAL, "bad precision");
    if (o->guess != GR_GUESS_ZERO && o->guess != GR_GUESS_CURRENT && o->guess != GR_GUESS_CHECKED)
        return fail(GR_EINVAL, "bad guess mode");
    return GR_OK;
}

int check_bound(gr_grid g)
{
    if (!g) return fail(GR_EINVAL, "null grid");
    if (!g->bound) return fail(GR_ESTATE, "grid not bound to a workspace");
    return GR_OK;
}

double *slot_ptr(gr_grid g, int field)
{
    if (field >= 0 && field < 10) return g->field[field];
    if (field >= GR_S0 && field <= GR_SM) return g->src[field - GR_S0];
    if (field == GR_AA) return g->AA;
    if (field == GR_RHS) return g->lev[0].f;
    if (field == GR_COEF) return g->lev[0].coef;
    if (field >= GR_HIST && field < GR_HIST + 10 && !g->solver_only) return g->hist[field - GR_HIST];
    return nullptr;
}

} // namespace

// ================================================ allocation-free single solve
//
// Scratch of gr_solve_equation_static: one file-scope device array per GPU
// (each device holds its own copy at its own address) that carries the level
// hierarchy of one solver-only grid of side <= kStaticMaxN.  Host code never
// passes the array's name to a kernel: its device address is taken once per
// device with hipGetSymbolAddress and kept in StaticDev::ptr.

namespace {
constexpr size_t kStaticScratchBytes = size_t(16) << 20; // levels of a 64^3 grid, FP64 and FP32
constexpr int kStaticMaxN = 64;
constexpr int kStaticMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct StaticDev {
    std::mutex mu;         // serialises the calls on one device within the process
    char *ptr = nullptr;   // device address of `scratch` on this device
    gr_grid_s grid;        // host-side description carved over the scratch
};
StaticDev g_static[kStaticMaxDevices];
} // namespace

// ===================================================================== ABI

namespace {
struct TuneEntry {
    int n, kind;
    FusedCfg cfg;
    float us;
    bool split;
};
std::vector<TuneEntry> g_tune_cache;
std::mutex g_tune_mu;
} // namespace

extern "C" {

const char *gr_last_error(void) { return g_err.c_str(); }

int gr_default_opts(gr_solve_opts *o)
{
    if (!o) return fail(GR_EINVAL, "null opts");
    o->nu1 = 2;
    o->nu2 = 2;
    o->max_cycles = 100;
    o->rtol = 1e-10;
    o->precision = GR_FP64;
    o->guess = GR_GUESS_ZERO;
    o->field_mask = GR_ALL_FIELDS;
    return GR_OK;
}

int gr_create_grid(const gr_grid_desc *desc, const gr_params *prm, gr_grid *out)
{
    if (!desc || !prm || !out) return fail(GR_EINVAL, "null argument");
    *out = nullptr;
    const int n = desc->n;
    if (n < 2 || (n & 1) || n > 1024) return fail(GR_EINVAL, "n = %d must be even, 2..1024", n);
    if (!(desc->h > 0.0) || !std::isfinite(desc->h)) return fail(GR_EINVAL, "h must be positive");
    if (!(prm->a > 0.0) || !(prm->c_tilde > 0.0) || !std::isfinite(prm->omega_m))
        return fail(GR_EINVAL, "a and c_tilde must be positive");
    gr_grid g = new (std::nothrow) gr_grid_s();
    if (!g) return fail(GR_EINVAL, "out of host memory");
    g->n = n;
    g->h = desc->h;
    g->prm = *prm;
    g->nlev = num_levels(n);
    // tuning knobs (environment): GRMG_SMOOTHER=split|fused forces one smoother
    // on every level it can run on; GRMG_FUSED_MIN (smallest level for the fused
    // smoother), GRMG_FUSED_TILE (0: 64x8, 1: 32x16, 2: 64x16, 3: 128x8), GRMG_XCD_REMAP (0/1/2),
    // GRMG_FUSED_WGS (target workgroups per fused launch), GRMG_FUSED_PF (prefetch
    // depth 1 to 4 planes), GRMG_COARSE_N (levels
    // at or below this size run the rest of the V-cycle in one workgroup; 0: never;
    // GRMG_COARSE_N32 likewise for the FP32 correction cycles; GRMG_COARSE_NP the
    // same for the Poisson kind in both, 16 by default),
    // GRMG_MIXED_STALL (mixed-precision stagnation ratio), GRMG_GRAPH (0: launch
    // every cycle's kernels one by one instead of replaying a captured graph)
    if (const char *e = std::getenv("GRMG_SMOOTHER")) {
        g->fused = std::strcmp(e, "split") != 0;
        if (std::strcmp(e, "fused") == 0) g->fcfg.min_n = 64;
    }
    if (const char *e = std::getenv("GRMG_FUSED_MIN")) g->fcfg.min_n = std::atoi(e);
    if (const char *e = std::getenv("GRMG_FUSED_TILE")) g->fcfg.tile = std::min(3, std::max(0, std::atoi(e)));
    if (const char *e = std::getenv("GRMG_XCD_REMAP")) g->fcfg.xcd_remap = std::atoi(e);
    if (const char *e = std::getenv("GRMG_FUSED_WGS")) g->fcfg.target_wgs = std::max(1, std::atoi(e));
    if (const char *e = std::getenv("GRMG_FUSED_PF")) g->fcfg.pf = std::min(4, std::max(0, std::atoi(e)));
    if (const char *e = std::getenv("GRMG_COARSE_N")) g->coarse_n = std::atoi(e);
    if (const char *e = std::getenv("GRMG_COARSE_N32")) g->coarse_n32 = std::atoi(e);
    if (const char *e = std::getenv("GRMG_COARSE_NP")) g->coarse_np = std::atoi(e);
    if (const char *e = std::getenv("GRMG_MIXED_STALL")) g->stall_ratio = std::atof(e);
    if (const char *e = std::getenv("GRMG_GRAPH")) g->use_graph = std::atoi(e) != 0;
    if (const char *e = std::getenv("GRMG_SKEW")) g->skew = std::max(0, std::atoi(e));
    if (g->nlev > kMaxLevels) {
        delete g;
        return fail(GR_EINVAL, "too many levels");
    }
    for (int l = 0; l < g->nlev; ++l) {
        g->lev[l].n = n >> l;
        g->lev[l].h = desc->h * (double)(1 << l);
        g->lev[l].N = (long)g->lev[l].n * g->lev[l].n * g->lev[l].n;
    }
    // GRMG_CONCURRENT=0: solve the components of vector equations one after another
    bool conc = n >= 64;
    if (const char *e = std::getenv("GRMG_CONCURRENT")) conc = conc && std::atoi(e) != 0;
    if (conc)
        for (auto &h : g->sub) {
            h = new (std::nothrow) gr_grid_s();
            if (!h) {
                delete g;
                return fail(GR_EINVAL, "out of host memory");
            }
            h->solver_only = true;
            h->n = g->n;
            h->h = g->h;
            h->prm = g->prm;
            h->nlev = g->nlev;
            for (int l = 0; l < g->nlev; ++l) {
                h->lev[l].n = g->lev[l].n;
                h->lev[l].h = g->lev[l].h;
                h->lev[l].N = g->lev[l].N;
            }
            h->fused = g->fused;
            h->fcfg = g->fcfg;
            h->coarse_n = g->coarse_n;
            h->coarse_n32 = g->coarse_n32;
            h->coarse_np = g->coarse_np;
            h->stall_ratio = g->stall_ratio;
            h->use_graph = g->use_graph;
            h->skew = g->skew;
        }
    g->ws_bytes = layout(g, nullptr);
    *out = g;
    return GR_OK;
}

int gr_workspace_bytes(gr_grid g, size_t *bytes)
{
    if (!g || !bytes) return fail(GR_EINVAL, "null argument");
    *bytes = g->ws_bytes;
    return GR_OK;
}

int gr_bind(gr_grid g, void *d_ws, size_t bytes, void *stream)
{
    if (!g || !d_ws) return fail(GR_EINVAL, "null argument");
    if (bytes < g->ws_bytes) return fail(GR_EINVAL, "workspace %zu bytes < required %zu", bytes, g->ws_bytes);
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(GR_EINVAL, "workspace not 256-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_ws) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(GR_EINVAL, "workspace is not device memory");
    }
    g->user_stream = reinterpret_cast<hipStream_t>(stream);
    g->stream = g->user_stream;
    g->drop_graphs();
    if (!g->work) {
        HIPCHK(hipStreamCreateWithFlags(&g->work, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&g->ev_norms, hipEventDisableTiming));
        HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&g->h_norms), 2 * sizeof(double),
                             hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void **>(&g->d_norms), g->h_norms, 0));
    }
    for (auto *h : g->sub) {
        if (!h) continue;
        h->drop_graphs();
        if (!h->work) {
            HIPCHK(hipStreamCreateWithFlags(&h->work, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->ev_norms, hipEventDisableTiming));
            HIPCHK(hipHostMalloc(reinterpret_cast<void **>(&h->h_norms), 2 * sizeof(double),
                                 hipHostMallocMapped | hipHostMallocCoherent));
            HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void **>(&h->d_norms), h->h_norms, 0));
        }
        h->user_stream = g->user_stream;
        h->stream = g->user_stream;
        h->bound = true;
    }
    layout(g, reinterpret_cast<char *>(d_ws));
    for (int f = 0; f < 10; ++f) g->alt_valid[f] = g->hist_valid[f] = false;
    launch_fill(g->stream, reinterpret_cast<double *>(d_ws), (long)(g->ws_bytes / sizeof(double)), 0.0);
    LAUNCHCHK();
    g->bound = true;
    return GR_OK;
}

int gr_destroy_grid(gr_grid g)
{
    delete g;
    return GR_OK;
}

int gr_deposit_sources(gr_grid g, const double *d_pos, const double *d_u, double mass, int64_t np)
{
    CHK(check_bound(g));
    if (np < 0 || (np > 0 && (!d_pos || !d_u))) return fail(GR_EINVAL, "bad particle arrays");
    if (!std::isfinite(mass)) return fail(GR_EINVAL, "mass not finite");
    const long N = g->N();
    if (np <= N) {
        launch_cic_sorted(g->stream, g->n, g->prm.a, g->prm.c_tilde, d_pos, d_u, mass, (long)np, g->field[GR_PSI],
                          g->cic, g->src[0], g->src[1], g->src[2], g->src[3], g->src[4]);
    } else { // more particles than cells: scatter with floating-point atomics
        for (int c = 0; c < 5; ++c) launch_fill(g->stream, g->src[c], N, 0.0);
        launch_cic_deposit(g->stream, g->n, g->prm.a, g->prm.c_tilde, d_pos, d_u, mass, (long)np,
                           g->field[GR_PSI], g->src[0], g->src[1], g->src[2], g->src[3], g->src[4]);
    }
    LAUNCHCHK();
    return GR_OK;
}

// Phi (into the scratch A6[0]) and beta^i (A6[1..3]) from the held fields, for
// the particle calls; A_ij is rebuilt by the next solve.
namespace {
int particle_metric(gr_grid g, const double **Phi, const double *beta[3])
{
    const double a = g->prm.a, c = g->prm.c_tilde;
    launch_derived(g->stream, 0, g->A6[0], g->field[GR_PSI], g->field[GR_XI], nullptr, nullptr, g->n, g->h, a, c);
    for (int d = 0; d < 3; ++d)
        launch_derived(g->stream, 3 + d, g->A6[1 + d], g->field[GR_PSI], g->field[GR_XI], g->field[GR_BX + d],
                       g->field[GR_BB], g->n, g->h, a, c);
    LAUNCHCHK();
    *Phi = g->A6[0];
    for (int d = 0; d < 3; ++d) beta[d] = g->A6[1 + d];
    return GR_OK;
}

int check_particles(gr_grid g, const void *pos, const void *u, int64_t np, double dt)
{
    CHK(check_bound(g));
    if (np < 0 || (np > 0 && (!pos || !u))) return fail(GR_EINVAL, "bad particle arrays");
    if (!std::isfinite(dt)) return fail(GR_EINVAL, "dt not finite");
    if (std::fabs(g->h * g->n - 1.0) > 1e-12) return fail(GR_EINVAL, "particles need the unit box (h = 1/n)");
    return GR_OK;
}
} // namespace

int gr_kick(gr_grid g, const double *d_pos, double *d_u, int64_t np, double dt, int order)
{
    CHK(check_particles(g, d_pos, d_u, np, dt));
    if (order != GR_KICK_FORWARD && order != GR_KICK_REVERSE) return fail(GR_EINVAL, "bad kick order %d", order);
    const double *Phi = nullptr, *beta[3];
    CHK(particle_metric(g, &Phi, beta));
    launch_kick(g->stream, g->n, g->prm.a, g->prm.c_tilde, Phi, g->field[GR_PSI], beta, d_pos, d_u, (long)np, dt,
                order);
    LAUNCHCHK();
    return GR_OK;
}

int gr_drift(gr_grid g, double *d_pos, const double *d_u, int64_t np, double dt)
{
    CHK(check_particles(g, d_pos, d_u, np, dt));
    const double *Phi = nullptr, *beta[3];
    CHK(particle_metric(g, &Phi, beta));
    launch_drift(g->stream, g->n, g->prm.a, g->prm.c_tilde, Phi, g->field[GR_PSI], beta, d_pos, d_u, (long)np, dt);
    LAUNCHCHK();
    return GR_OK;
}

int gr_newtonian_kick(gr_grid g, const double *d_pos, double *d_u, int64_t np, double dt, const gr_solve_opts *opts,
                      gr_solve_report *rep)
{
    g_err.clear();
    CHK(check_particles(g, d_pos, d_u, np, dt));
    CHK(check_opts(opts));
    if (opts->guess == GR_GUESS_CHECKED) return fail(GR_EINVAL, "the Newtonian potential starts from zero");
    WorkScope ws(g);
    if (!ws.ok) return fail(GR_EDEVICE, "cannot join the work stream");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const long N = g->N();
    double *phiN = g->A6[5]; // scratch until the next solve rebuilds A_ij
    // Lap Phi_N = 3/2 a Om (s0 - <s0>) for periodic solvability, formed as
    // 3/2 a Om (s0 - 1) minus its own mean (no cancellation of the mean against 1)
    launch_ham_rhs(s, g->lev[0].f, g->src[0], N, 1.5 * g->prm.a * g->prm.omega_m);
    CHK(reduce_mean(g, g->lev[0].f, nullptr, N, g->scal + S_SCRATCH));
    launch_sub_scalar(s, g->lev[0].f, N, g->scal + S_SCRATCH);
    launch_fill(s, phiN, N, 0.0);
    LAUNCHCHK();
    int cyc = 0, fb = 0;
    double rel = 0.0;
    int st = solve_field(g, GR_KIND_POISSON, phiN, *opts, &cyc, &rel, &fb);
    if (st == GR_EDEVICE) return st;
    launch_newton_kick(s, g->n, phiN, d_pos, d_u, (long)np, dt);
    LAUNCHCHK();
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(GR_EDEVICE, "sync: %s", hipGetErrorString(e));
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->status = st;
        rep->cycles[0] = cyc;
        rep->rel_res[0] = rel;
        rep->fallback = fb;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

int gr_set_field(gr_grid g, int field, const void *d_src, int dtype)
{
    CHK(check_bound(g));
    double *dst = slot_ptr(g, field);
    if (!dst) return fail(GR_EINVAL, "field %d cannot be set", field);
    if (field >= GR_HIST && field < GR_HIST + 10) g->hist_valid[field - GR_HIST] = true;
    if (!d_src) return fail(GR_EINVAL, "null source");
    if (dtype == GR_F64) launch_copy(g->stream, dst, static_cast<const double *>(d_src), g->N());
    else if (dtype == GR_F32) launch_convert_f32_to_f64(g->stream, dst, static_cast<const float *>(d_src), g->N());
    else return fail(GR_EINVAL, "bad dtype %d", dtype);
    LAUNCHCHK();
    return GR_OK;
}

int gr_get_field(gr_grid g, int field, void *d_dst, int dtype)
{
    CHK(check_bound(g));
    if (!d_dst) return fail(GR_EINVAL, "null destination");
    if (dtype != GR_F64 && dtype != GR_F32) return fail(GR_EINVAL, "bad dtype %d", dtype);
    const long N = g->N();
    const double *srcp = slot_ptr(g, field);
    double *tmp = g->lev[0].tmp;
    if (!srcp) {
        if (field < GR_PHI || field > GR_BETAZ) return fail(GR_EINVAL, "unknown field %d", field);
        const int which = field - GR_PHI; // 0 Phi, 1 alpha, 2 psi, 3..5 beta
        const double *Bc = which >= 3 ? g->field[GR_BX + (which - 3)] : nullptr;
        double *out = dtype == GR_F64 ? static_cast<double *>(d_dst) : tmp;
        launch_derived(g->stream, which, out, g->field[GR_PSI], g->field[GR_XI], Bc, g->field[GR_BB], g->n, g->h,
                       g->prm.a, g->prm.c_tilde);
        if (dtype == GR_F32) launch_convert_f64_to_f32(g->stream, static_cast<float *>(d_dst), tmp, N);
        LAUNCHCHK();
        return GR_OK;
    }
    if (dtype == GR_F64) launch_copy(g->stream, static_cast<double *>(d_dst), srcp, N);
    else launch_convert_f64_to_f32(g->stream, static_cast<float *>(d_dst), srcp, N);
    LAUNCHCHK();
    return GR_OK;
}

int gr_solve_equation(gr_grid g, int kind, int field, const gr_solve_opts *opts, gr_solve_report *rep)
{
    g_err.clear();
    CHK(check_bound(g));
    CHK(check_opts(opts));
    if (kind < 0 || kind > 2) return fail(GR_EINVAL, "bad kind %d", kind);
    if (field < 0 || field > 9) return fail(GR_EINVAL, "bad field %d", field);
    WorkScope ws(g);
    if (!ws.ok) return fail(GR_EDEVICE, "cannot join the work stream");
    auto t0 = std::chrono::steady_clock::now();
    if (opts->guess == GR_GUESS_ZERO) launch_fill(g->stream, g->field[field], g->N(), 0.0);
    int cyc = 0;
    double rel = 0.0;
    int fb = 0;
    int st = solve_field(g, kind, g->field[field], *opts, &cyc, &rel, &fb);
    if (st != GR_EDEVICE) {
        hipError_t e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) st = fail(GR_EDEVICE, "sync: %s", hipGetErrorString(e));
    }
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->status = st;
        rep->cycles[0] = cyc;
        rep->rel_res[0] = rel;
        rep->fallback = fb;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

int gr_solve_equation_static(int n, const gr_params *prm, int kind, const double *d_f, const double *d_coef,
                             double *d_phi, const gr_solve_opts *opts, void *hip_stream, gr_solve_report *rep)
{
    g_err.clear();
    if (!prm || !d_f || !d_phi || !opts) return fail(GR_EINVAL, "null argument");
    if (kind < 0 || kind > 2) return fail(GR_EINVAL, "bad kind %d", kind);
    if (kind != GR_KIND_POISSON && !d_coef) return fail(GR_EINVAL, "kind %d needs a coefficient array", kind);
    if (n < 2 || (n & 1) || n > kStaticMaxN)
        return fail(GR_EINVAL, "n = %d: the allocation-free solve takes even n from 2 to %d (%zu-byte static scratch)",
                    n, kStaticMaxN, kStaticScratchBytes);
    if (!(prm->a > 0.0) || !(prm->c_tilde > 0.0) || !std::isfinite(prm->omega_m))
        return fail(GR_EINVAL, "a and c_tilde must be positive");
    CHK(check_opts(opts));
    if (opts->guess == GR_GUESS_CHECKED) return fail(GR_EINVAL, "no saved alternative guess here: use ZERO or CURRENT");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticMaxDevices) return fail(GR_EINVAL, "device %d beyond %d", dev, kStaticMaxDevices);
    StaticDev &S = g_static[dev];
    std::lock_guard<std::mutex> lock(S.mu);
    if (!S.ptr) { // once per device, with that device current
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GR_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        S.ptr = static_cast<char *>(p);
    }
    auto t0 = std::chrono::steady_clock::now();
    // a solver-only grid with the library's default launch choices, no
    // private stream and no captured graphs (instantiating one allocates)
    gr_grid g = &S.grid;
    g->solver_only = true;
    g->n = n;
    g->h = 1.0 / n;
    g->prm = *prm;
    g->nlev = num_levels(n);
    for (int l = 0; l < kMaxLevels; ++l) g->lev[l] = Level{};
    for (int l = 0; l < g->nlev; ++l) {
        g->lev[l].n = n >> l;
        g->lev[l].h = g->h * (double)(1 << l);
        g->lev[l].N = (long)g->lev[l].n * g->lev[l].n * g->lev[l].n;
    }
    g->fused = true;
    g->fcfg = FusedCfg{};
    std::memset(g->tuned_ok, 0, sizeof g->tuned_ok);
    std::memset(g->tuned_split, 0, sizeof g->tuned_split);
    g->coarse_n = 8;
    g->coarse_n32 = 8;
    g->coarse_np = 16;
    g->skew = 0;
    g->stall_ratio = 0.5;
    g->use_graph = false;
    g->timing = false;
    g->sub[0] = g->sub[1] = nullptr;
    g->h_norms = nullptr; // read-back waits on the stream (pinned slots would be an allocation)
    g->ev_norms = nullptr;
    const size_t need = layout(g, nullptr);
    if (need > kStaticScratchBytes)
        return fail(GR_EINVAL, "n = %d needs %zu bytes of scratch, more than %zu", n, need, kStaticScratchBytes);
    layout(g, S.ptr);
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    g->user_stream = g->stream = s;
    g->work = nullptr;
    g->bound = true;
    // the array keeps the previous call's contents: start from zeros, as a bind does
    launch_fill(s, reinterpret_cast<double *>(S.ptr), (long)(need / sizeof(double)), 0.0);
    const long N = g->N();
    launch_copy(s, g->lev[0].f, d_f, N);
    if (kind != GR_KIND_POISSON) launch_copy(s, g->lev[0].coef, d_coef, N);
    if (opts->guess == GR_GUESS_ZERO) launch_fill(s, d_phi, N, 0.0);
    LAUNCHCHK();
    int cyc = 0, fb = 0;
    double rel = 0.0;
    int st = solve_field(g, kind, d_phi, *opts, &cyc, &rel, &fb);
    if (st != GR_EDEVICE) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(GR_EDEVICE, "sync: %s", hipGetErrorString(e));
    }
    g->bound = false;
    if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->status = st;
        rep->cycles[0] = cyc;
        rep->rel_res[0] = rel;
        rep->fallback = fb;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

int gr_solve_constraints(gr_grid g, const gr_solve_opts *opts, gr_solve_report *rep)
{
    g_err.clear(); // a message left by an earlier call must not be reported for this one
    CHK(check_bound(g));
    CHK(check_opts(opts));
    WorkScope ws(g);
    if (!ws.ok) return fail(GR_EDEVICE, "cannot join the work stream");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const long N = g->N();
    const double a = g->prm.a, om = g->prm.omega_m, c = g->prm.c_tilde;
    const unsigned mask = opts->field_mask;
    gr_solve_report R;
    std::memset(&R, 0, sizeof R);
    int first_bad = GR_OK;
    if (opts->guess == GR_GUESS_ZERO)
        for (int f = 0; f < 10; ++f)
            if (mask & (1u << f)) {
                launch_fill(s, g->field[f], N, 0.0);
                g->hist_valid[f] = false; // a solve from zero starts a new trajectory
            }
    LAUNCHCHK();
    double *fine_f = g->lev[0].f;
    double *fine_c = g->lev[0].coef;

    auto solve = [&](int fid, int kind) -> int {
        if (!(mask & (1u << fid))) return GR_OK;
        if (opts->guess == GR_GUESS_CHECKED) {
            int took = 0;
            CHK(choose_guess(g, kind, fid, &took, &R.guess_rel[fid], &R.alt_rel[fid]));
            R.guess_fallback += took;
        }
        g->alt_valid[fid] = false; // a saved alternative serves one solve only
        int fb = 0;
        int st = solve_field(g, kind, g->field[fid], *opts, &R.cycles[fid], &R.rel_res[fid], &fb);
        R.fallback += fb;
        if (st == GR_EDEVICE) return st;
        if (st != GR_OK && first_bad == GR_OK) first_bad = st;
        return GR_OK;
    };

    // The three components of a vector equation: with helper hierarchies, each
    // component's solve runs on its own stream and host thread (the small,
    // latency-bound levels of the three V-cycles overlap); build(d, f) writes
    // component d's source on this grid's stream.
    auto solve3 = [&](int fid0, const std::function<int(int, double *)> &build) -> int {
        gr_grid H[3] = {g, g->sub[0], g->sub[1]};
        if (!g->sub[0] || !g->sub[1]) {
            for (int d = 0; d < 3; ++d) {
                if (!(mask & (1u << (fid0 + d)))) continue;
                CHK(build(d, fine_f));
                CHK(solve(fid0 + d, GR_KIND_POISSON));
            }
            return GR_OK;
        }
        for (int d = 0; d < 3; ++d)
            if (mask & (1u << (fid0 + d))) CHK(build(d, H[d]->lev[0].f));
        for (int d = 1; d < 3; ++d) { // helpers start after the sources
            HIPCHK(hipEventRecord(H[d]->ev_in, s));
            HIPCHK(hipStreamWaitEvent(H[d]->work, H[d]->ev_in, 0));
            H[d]->stream = H[d]->work;
        }
        struct Out {
            int st = GR_OK, cyc = 0, fb = 0, took = 0;
            double rel = 0.0, grel = 0.0, arel = 0.0;
            std::string err;
        } out[3];
        auto run = [&](int d) {
            const int fid = fid0 + d;
            if (!(mask & (1u << fid))) return;
            gr_grid h = H[d];
            Out &o = out[d];
            o.st = [&]() -> int {
                if (opts->guess == GR_GUESS_CHECKED)
                    CHK(choose_guess_on(h, GR_KIND_POISSON, g->field[fid], g->alt[fid], g->alt_valid[fid], &o.took,
                                        &o.grel, &o.arel));
                return solve_field(h, GR_KIND_POISSON, g->field[fid], *opts, &o.cyc, &o.rel, &o.fb);
            }();
            if (o.st != GR_OK) o.err = g_err;
        };
        std::thread t1(run, 1), t2(run, 2);
        run(0);
        t1.join();
        t2.join();
        for (int d = 1; d < 3; ++d) { // this grid's stream waits for the helpers
            (void)hipEventRecord(H[d]->ev_out, H[d]->work);
            (void)hipStreamWaitEvent(s, H[d]->ev_out, 0);
            H[d]->stream = H[d]->user_stream;
        }
        int dev = GR_OK;
        for (int d = 0; d < 3; ++d) {
            const int fid = fid0 + d;
            if (!(mask & (1u << fid))) continue;
            const Out &o = out[d];
            R.cycles[fid] = o.cyc;
            R.rel_res[fid] = o.rel;
            R.fallback += o.fb;
            R.guess_fallback += o.took;
            R.guess_rel[fid] = o.grel;
            R.alt_rel[fid] = o.arel;
            g->alt_valid[fid] = false;
            if (o.st != GR_OK) {
                g_err = o.err;
                if (o.st == GR_EDEVICE) dev = GR_EDEVICE;
                else if (first_bad == GR_OK) first_bad = o.st;
            }
        }
        return dev;
    };

    // 1. V_i: Lap V_i = 3 Om a (s_i - <s_i>)
    CHK(solve3(GR_VX, [&](int d, double *f) -> int {
        CHK(reduce_mean(g, g->src[1 + d], nullptr, N, g->scal + S_SCRATCH + d));
        launch_shift_scale(s, f, g->src[1 + d], N, 3.0 * om * a, g->scal + S_SCRATCH + d);
        LAUNCHCHK();
        return GR_OK;
    }));
    // 2. U: Lap U = -1/4 d_j V^j
    launch_div_quarter(s, fine_f, g->field[GR_VX], g->field[GR_VY], g->field[GR_VZ], g->n, g->h);
    LAUNCHCHK();
    CHK(solve(GR_U, GR_KIND_POISSON));
    // 3. A_ij and AA
    launch_build_Aij(s, g->A6, g->AA, g->field[GR_VX], g->field[GR_VY], g->field[GR_VZ], g->field[GR_U], g->n, g->h);
    // 4. Psi: f = 3/2 a Om (s0 - 1), coefficient AA
    launch_ham_rhs(s, fine_f, g->src[0], N, 1.5 * a * om);
    launch_copy(s, fine_c, g->AA, N);
    LAUNCHCHK();
    CHK(solve(GR_PSI, GR_KIND_HAMILTONIAN));
    // 5. xi: CMC with m2 and f from the solved Psi
    launch_build_cmc(s, fine_c, fine_f, g->field[GR_PSI], g->src[0], g->src[4], g->AA, N, a, om, c);
    LAUNCHCHK();
    CHK(solve(GR_XI, GR_KIND_CMC));
    // 6. B^i: Lap B^i = 2 d_j[alpha chi^-6 A^ij]
    launch_shift_source(s, g->fB, g->field[GR_PSI], g->field[GR_XI], g->A6, g->n, g->h, a, c);
    LAUNCHCHK();
    CHK(solve3(GR_BX, [&](int d, double *f) -> int {
        launch_copy(s, f, g->fB[d], N);
        LAUNCHCHK();
        return GR_OK;
    }));
    // 7. b: Lap b = -1/4 d_j B^j
    launch_div_quarter(s, fine_f, g->field[GR_BX], g->field[GR_BY], g->field[GR_BZ], g->n, g->h);
    LAUNCHCHK();
    CHK(solve(GR_BB, GR_KIND_POISSON));
    HIPCHK(hipStreamSynchronize(s));
    R.status = first_bad;
    R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = R;
    if (first_bad != GR_OK && g_err.empty()) fail(first_bad, "a field did not converge");
    return first_bad;
}

int gr_features(gr_grid g, int level, int count, const int *fields, const double *offset, const double *scale,
                float *d_dst, int flags)
{
    CHK(check_bound(g));
    if (level < 0 || level >= g->nlev || count < 1 || count > 32 || !fields || !offset || !scale || !d_dst ||
        (flags & ~GR_FEAT_ACCUMULATE))
        return fail(GR_EINVAL, "bad argument");
    for (int c = 0; c < count; ++c)
        if (!slot_ptr(g, fields[c]) || fields[c] == GR_RHS || fields[c] == GR_COEF)
            return fail(GR_EINVAL, "field %d", fields[c]);
    hipStream_t s = g->stream;
    const long M = g->lev[level].N;
    for (int c = 0; c < count; ++c) {
        const double *src = slot_ptr(g, fields[c]);
        for (int l = 1; l <= level; ++l) {
            launch_restrict(s, src, g->lev[l - 1].n, g->lev[l].tmp);
            src = g->lev[l].tmp;
        }
        launch_affine_to_f32(s, d_dst + c * M, src, M, offset[c], scale[c], (flags & GR_FEAT_ACCUMULATE) != 0);
    }
    LAUNCHCHK();
    return GR_OK;
}

int gr_set_guess(gr_grid g, int level, int count, const int *fields, const double *scale, const float *d_src,
                 int flags)
{
    CHK(check_bound(g));
    if (level < 0 || level >= g->nlev || count < 1 || count > 10 || !fields || !scale || !d_src ||
        (flags & ~(GR_SET_ADD | GR_SET_CUBIC | GR_SET_EXTRAP)))
        return fail(GR_EINVAL, "bad argument");
    for (int c = 0; c < count; ++c)
        if (fields[c] < 0 || fields[c] > 9) return fail(GR_EINVAL, "field %d is not a solved field", fields[c]);
    hipStream_t s = g->stream;
    const long N = g->N();
    const long M = g->lev[level].N;
    for (int c = 0; c < count; ++c) {
        const int f = fields[c];
        // prediction (times scale) into level `level`, then interpolated level by level to the finest
        double *cur = g->lev[level].tmp;
        launch_f32_scaled_to_f64(s, cur, d_src + c * M, M, scale[c]);
        for (int l = level; l >= 1; --l) {
            Level &C = g->lev[l], &F = g->lev[l - 1];
            if (flags & GR_SET_CUBIC) {
                const int m = C.n;
                double *X = g->gtmp, *Y = g->gtmp + N / 4; // (m,m,2m) then (m,2m,2m)
                launch_cubic_pass(s, cur, m, m, m, 0, X);
                launch_cubic_pass(s, X, 2 * m, m, m, 1, Y);
                launch_cubic_pass(s, Y, 2 * m, 2 * m, m, 2, F.tmp);
            } else {
                launch_fill(s, C.phi0, C.N, 0.0);
                launch_fill(s, F.tmp, F.N, 0.0);
                launch_prolong_correct(s, F.tmp, F.n, cur, C.phi0);
            }
            cur = F.tmp;
        }
        if (flags & GR_SET_EXTRAP) {
            // held f (previous step), history h (the step before): field = (2f - h) + P pred,
            // or f + P pred without a history; then history and alternative = f
            launch_extrapolate(s, g->field[f], g->hist[f], g->alt[f], cur, g->hist_valid[f], N);
            g->hist_valid[f] = true;
            g->alt_valid[f] = true;
        } else if (flags & GR_SET_ADD) {
            launch_copy(s, g->alt[f], g->field[f], N);
            g->alt_valid[f] = true;
            launch_axpy(s, g->field[f], cur, N);
        } else {
            launch_copy(s, g->field[f], cur, N);
            g->alt_valid[f] = false;
        }
    }
    LAUNCHCHK();
    return GR_OK;
}

// Autotuner of the fused sweep: for every fused level and kind, time each
// candidate (tile shape x workgroup target x prefetch depth) on scratch
// arrays and keep the fastest.  Results are cached per process by (n, kind)
// so later grids of the same size reuse them.  The sweep's result does not
// depend on the configuration (same per-point arithmetic, exact red-black
// order), only its speed does.

const char *const kTileName[4] = {"64x8", "32x16", "64x16", "128x8"};

int gr_autotune(gr_grid g, char *report, size_t report_bytes)
{
    CHK(check_bound(g));
    WorkScope ws(g);
    if (!ws.ok) return fail(GR_EDEVICE, "cannot join the work stream");
    hipStream_t s = g->stream;
    std::string rep;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const OpConst oc = g->oc();
    const double *zero = g->scal + S_ZERO;
    int st = GR_OK;
    for (int l = 0; l < g->nlev && st == GR_OK; ++l) {
        const Level &L = g->lev[l];
        // every level the fused sweep can tile (the size threshold is for untuned grids)
        if (!g->fused || !fused_sweep_ok(L.n, 32)) continue;
        const long M = L.N;
        double *d = static_cast<double *>(g->cic); // scratch: 8 n^3 doubles
        float *fl = static_cast<float *>(g->cic);
        for (int kind = 0; kind < 6 && st == GR_OK; ++kind) {
            FusedCfg best = g->fcfg;
            float best_us = -1.f;
            bool split = false;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                for (auto &e : g_tune_cache)
                    if (e.n == L.n && e.kind == kind) {
                        best = e.cfg;
                        best_us = e.us;
                        split = e.split;
                    }
            }
            if (best_us < 0.f) {
                for (int tile = 0; tile < (L.n % 128 == 0 ? 4 : 3); ++tile)
                    for (int wgs : {256, 512, 1024, 2048})
                        if (L.n % 64 == 0 || tile == 1) // 32 x 16 only where 64-wide tiles do not fit
                        for (int pf = 1; pf <= (tile == 2 ? 4 : 2); ++pf) {
                            FusedCfg c = g->fcfg;
                            c.tile = tile;
                            c.target_wgs = wgs;
                            c.pf = pf;
                            auto sweep = [&]() {
                                if (kind < 3)
                                    launch_rb_fused(kind, s, d, d + M, d + 2 * M, d + 3 * M, L.n, L.h, oc, zero,
                                                    zero, c);
                                else
                                    launch_rb_fused_f32(kind, s, fl, fl + M, fl + 2 * M, fl + 3 * M, fl + 4 * M, L.n,
                                                        L.h, oc, zero, c);
                            };
                            sweep();
                            (void)hipEventRecord(e0, s);
                            for (int r = 0; r < 4; ++r) sweep();
                            (void)hipEventRecord(e1, s);
                            hipError_t he = hipEventSynchronize(e1);
                            if (he != hipSuccess) {
                                st = fail(GR_EDEVICE, "autotune: %s", hipGetErrorString(he));
                                break;
                            }
                            float ms = 0.f;
                            (void)hipEventElapsedTime(&ms, e0, e1);
                            const float us = ms * 1e3f / 4.f;
                            if (best_us < 0.f || us < best_us) {
                                best_us = us;
                                best = c;
                            }
                        }
                if (st != GR_OK) break;
                { // one in-place launch per colour, for comparison
                    auto sweep = [&]() {
                        if (kind < 3)
                            launch_rb_sweep(kind, s, d, d + 2 * M, d + 3 * M, L.n, L.h, oc, zero, zero);
                        else
                            launch_rb_sweep_f32(kind, s, fl, fl + 2 * M, fl + 3 * M, fl + 4 * M, L.n, L.h, oc, zero);
                    };
                    sweep();
                    (void)hipEventRecord(e0, s);
                    for (int r = 0; r < 4; ++r) sweep();
                    (void)hipEventRecord(e1, s);
                    hipError_t he = hipEventSynchronize(e1);
                    if (he != hipSuccess) {
                        st = fail(GR_EDEVICE, "autotune: %s", hipGetErrorString(he));
                        break;
                    }
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    const float us = ms * 1e3f / 4.f;
                    if (us < best_us) {
                        best_us = us;
                        split = true;
                    }
                }
                if (st != GR_OK) break;
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune_cache.push_back({L.n, kind, best, best_us, split});
            }
            g->tuned[l][kind] = best;
            g->tuned_ok[l][kind] = true;
            g->tuned_split[l][kind] = split;
            char line[160];
            if (split)
                std::snprintf(line, sizeof line, "n=%d kind=%d split us=%.2f\n", L.n, kind, best_us);
            else
                std::snprintf(line, sizeof line, "n=%d kind=%d tile=%s wgs=%d pf=%d us=%.2f\n", L.n, kind,
                              kTileName[best.tile], best.target_wgs, best.pf,
                              best_us);
            rep += line;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    LAUNCHCHK();
    g->drop_graphs(); // captured cycles hold the old launch shapes
    for (auto *h : g->sub)
        if (h) {
            std::memcpy(h->tuned, g->tuned, sizeof g->tuned);
            std::memcpy(h->tuned_ok, g->tuned_ok, sizeof g->tuned_ok);
            std::memcpy(h->tuned_split, g->tuned_split, sizeof g->tuned_split);
            h->drop_graphs();
        }
    if (report && report_bytes) {
        std::snprintf(report, report_bytes, "%s", rep.c_str());
    }
    return st;
}

int gr_sweep_timing(gr_grid g, int enable, double *ms_sum, int *count)
{
    CHK(check_bound(g));
    if (enable) {
        if (!g->timing) g->graph_saved = g->use_graph;
        for (auto &e : g->sweep_ev) {
            g->ev_free.push_back(e.a);
            g->ev_free.push_back(e.b);
        }
        g->sweep_ev.clear();
        g->timing = true;
        g->use_graph = false; // launches bracketed by events are issued one by one
        return GR_OK;
    }
    if (!ms_sum || !count) return fail(GR_EINVAL, "null output");
    for (int k = 0; k < 6; ++k) {
        ms_sum[k] = 0.0;
        count[k] = 0;
    }
    for (auto &e : g->sweep_ev) {
        HIPCHK(hipEventSynchronize(e.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e.a, e.b));
        ms_sum[e.kind] += ms;
        count[e.kind] += 1;
        g->ev_free.push_back(e.a);
        g->ev_free.push_back(e.b);
    }
    g->sweep_ev.clear();
    if (g->timing) g->use_graph = g->graph_saved;
    g->timing = false;
    return GR_OK;
}

int gr_debug_sweep(gr_grid g, int kind, int field, double Fbar, double fshift, int nsweeps)
{
    CHK(check_bound(g));
    if (kind < 0 || kind > 2 || field < 0 || field > 9 || nsweeps < 0) return fail(GR_EINVAL, "bad argument");
    hipStream_t s = g->stream;
    launch_set_scalar(s, g->scal + S_FBAR, Fbar);
    launch_set_scalar(s, g->scal + S_FSHIFT, fshift);
    Level &L = g->lev[0];
    L.phi = g->field[field];
    double *tmp = L.tmp;
    EqCtx E{kind, g->oc(), 0, 0};
    const int st = smooth(g, E, 0, nsweeps);
    if (L.phi != g->field[field]) { // odd number of launches: the result is in the scratch array
        launch_copy(s, g->field[field], L.phi, L.N);
        L.phi = g->field[field];
    }
    L.tmp = tmp;
    LAUNCHCHK();
    return st;
}

int gr_debug_residual(gr_grid g, int kind, int field, double Fbar, double fshift, double *d_out)
{
    CHK(check_bound(g));
    if (kind < 0 || kind > 2 || field < 0 || field > 9 || !d_out) return fail(GR_EINVAL, "bad argument");
    hipStream_t s = g->stream;
    launch_set_scalar(s, g->scal + S_FBAR, Fbar);
    launch_set_scalar(s, g->scal + S_FSHIFT, fshift);
    Level &F = g->lev[0];
    launch_residual(kind, s, g->field[field], F.f, F.coef, F.n, F.h, g->oc(), g->scal + S_FBAR, g->scal + S_FSHIFT,
                    d_out);
    LAUNCHCHK();
    return GR_OK;
}

} // extern "C"
